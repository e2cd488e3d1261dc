"""Seeded synthetic instances of the random-indefinite sparse QP family.

This module draws problem data only; it contains none of the solver's
arithmetic.  Both the CPU oracle and the GPU path (through its Python
binding) consume what it produces.

Problem form (paper, Section 2, eq. (qp)):

    min 1/2 x'Qx + c'x  s.t.  rl <= A x <= ru,  xl <= x <= xu

with equality rows (rl == ru) first and one-sided ``>=`` rows after them.

Recipe (random indefinite family, family code 4; the seeding convention
``default_rng(SeedSequence([seed, family]))`` follows the paper's
appendix on scenario generation):

1. ``x_gen ~ U(0, 1)^n``                 (a feasible point used only to build b)
2. R: ``k_r`` distinct uniform columns per row, values N(0, 1)
3. ``Q = R + R' + diag(d)``, ``d ~ N(-1, 1)``  (symmetric, indefinite)
4. A: ``k_a`` distinct uniform columns per row, values N(0, 1)
5. rows ``0 .. m//2 - 1`` are equalities with ``rl = ru = A x_gen``;
   the rest are ``A x >= A x_gen - U(0, 1)`` (``ru = +inf``)
6. ``xl = 0``, ``xu = 1``, ``c ~ N(0, 1)``
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

FAMILY_RANDOM_INDEFINITE = 4


def _distinct_columns(rng, rows, k, n):
    """Draw ``k`` distinct uniform column indices in [0, n) for each row.

    Rows that drew a repeated column are redrawn whole until every row is
    duplicate-free; the result is sorted within each row.
    """
    k = min(k, n)
    cols = np.sort(rng.integers(0, n, size=(rows, k), dtype=np.int64), axis=1)
    while k > 1:
        bad = np.nonzero((np.diff(cols, axis=1) == 0).any(axis=1))[0]
        if bad.size == 0:
            break
        cols[bad] = np.sort(
            rng.integers(0, n, size=(bad.size, k), dtype=np.int64), axis=1)
    return cols


def _csr_from_rows(cols, vals, shape):
    rows, k = cols.shape
    indptr = np.arange(0, rows * k + 1, k, dtype=np.int64)
    M = sp.csr_matrix((vals.reshape(-1), cols.reshape(-1), indptr), shape=shape)
    return M


def _canonical(M):
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    M.indptr = M.indptr.astype(np.int32)
    M.indices = M.indices.astype(np.int32)
    M.data = M.data.astype(np.float64)
    return M


def random_indefinite_qp(n, m, k_r, k_a, seed, instance=None):
    """One instance of the random-indefinite family.

    ``instance`` (optional) appends a third word to the seed sequence so that
    the members of a batch are independent streams.

    Returns a dict with CSR ``Q`` (n x n, symmetric, both triangles stored),
    CSR ``A`` (m x n), and dense ``c, xl, xu, rl, ru`` plus ``x_gen``.
    """
    words = [int(seed), FAMILY_RANDOM_INDEFINITE]
    if instance is not None:
        words.append(int(instance))
    rng = np.random.default_rng(np.random.SeedSequence(words))

    x_gen = rng.uniform(0.0, 1.0, size=n)

    r_cols = _distinct_columns(rng, n, k_r, n)
    r_vals = rng.standard_normal(size=r_cols.shape)
    d = rng.normal(-1.0, 1.0, size=n)
    R = _csr_from_rows(r_cols, r_vals, (n, n))
    Q = _canonical(R + R.T + sp.diags(d, format="csr"))

    if m > 0:
        a_cols = _distinct_columns(rng, m, k_a, n)
        a_vals = rng.standard_normal(size=a_cols.shape)
        A = _canonical(_csr_from_rows(a_cols, a_vals, (m, n)))
    else:
        A = _canonical(sp.csr_matrix((0, n)))

    m_e = m // 2
    ax = A @ x_gen
    slack = rng.uniform(0.0, 1.0, size=m - m_e)
    rl = np.empty(m)
    ru = np.empty(m)
    rl[:m_e] = ax[:m_e]
    ru[:m_e] = ax[:m_e]
    rl[m_e:] = ax[m_e:] - slack
    ru[m_e:] = np.inf

    c = rng.standard_normal(size=n)
    xl = np.zeros(n)
    xu = np.ones(n)
    return dict(n=n, m=m, Q=Q, A=A, c=c, xl=xl, xu=xu, rl=rl, ru=ru,
                x_gen=x_gen, seed=seed, instance=instance,
                k_r=k_r, k_a=k_a)


# Named workloads.  Densities: "small" and "medium" draw 5 entries per row
# of R (about 11 per row of Q) and 4 per row of A; "large" is sized to the
# stated totals of roughly 5M nonzeros in Q and 4M in A at n = 1M, i.e. 2
# per row of R and 8 per row of A.  "large_literal" keeps the small-case
# densities at n = 1M.
WORKLOADS = {
    "small": dict(n=1000, m=500, k_r=5, k_a=4),
    "medium": dict(n=100_000, m=50_000, k_r=5, k_a=4),
    "large": dict(n=1_000_000, m=500_000, k_r=2, k_a=8),
    "large_literal": dict(n=1_000_000, m=500_000, k_r=5, k_a=4),
}


def workload(name, seed):
    """Instance of a named workload (see ``WORKLOADS``)."""
    p = WORKLOADS[name]
    return random_indefinite_qp(p["n"], p["m"], p["k_r"], p["k_a"], seed)


def batch_sizes(seed, count=512, lo=200, hi=20000):
    """Sizes n_i ~ U{lo..hi} of a batch; instance i then uses
    ``random_indefinite_qp(n_i, n_i // 2, 5, 4, seed, instance=i)``."""
    rng = np.random.default_rng(
        np.random.SeedSequence([int(seed), FAMILY_RANDOM_INDEFINITE]))
    return rng.integers(lo, hi + 1, size=count)


def batch(seed, count=512, lo=200, hi=20000):
    sizes = batch_sizes(seed, count, lo, hi)
    return [random_indefinite_qp(int(ni), int(ni) // 2, 5, 4, seed, instance=i)
            for i, ni in enumerate(sizes)]


FAMILY_FLOW = 2


def flow_qp(seed, n_target=1_000_000):
    """Concave-cost multistage flow, after the paper's appendix on the
    million-variable models (flow family) and its scenario-distribution
    table: minimise sum_e (c_e f_e - alpha c_e / u_e f_e^2) subject to
    B f = b (node-arc incidence, one equality row per node) and
    0 <= f <= u.

    Network: L layers of width w; each of three carriers joins layer l to
    layer l+1 through its own seeded permutation of the w nodes, so there
    are n = 3 w (L-1) arcs and m = L w nodes.  Scenario draws (in this
    order): L in {4, 6, 8, 12, 16}, alpha ~ U(0.03, 0.24), base cost
    ~ U(0.05, 0.30), capacity ratio rho ~ U(1.05, 1.80), stage growth
    g ~ U(0, 0.12), carrier-cost ratio ~ U(1/(1-2 alpha) + 0.25,
    1/(1-2 alpha) + 2), reference-flow interval bounds ~ U(0.30, 1.00) and
    U(1.20, 3.00), then one reference flow h_k per carrier uniform in that
    interval.

    Readings where the description leaves the construction open: carrier k
    costs base * ratio^k * (1 + g)^l on stage l; every arc of carrier k
    carries the reference flow h_k and has capacity rho * h_k; b = B f0, so
    the reference flow f0 is feasible (it is returned as ``x0``, the
    model's frozen start).
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), FAMILY_FLOW]))
    L = int(rng.choice([4, 6, 8, 12, 16]))
    alpha = rng.uniform(0.03, 0.24)
    base = rng.uniform(0.05, 0.30)
    rho = rng.uniform(1.05, 1.80)
    growth = rng.uniform(0.0, 0.12)
    r0 = 1.0 / (1.0 - 2.0 * alpha)
    ratio = rng.uniform(r0 + 0.25, r0 + 2.0)
    h_lo = rng.uniform(0.30, 1.00)
    h_hi = rng.uniform(1.20, 3.00)
    h = rng.uniform(h_lo, h_hi, size=3)
    w = max(1, n_target // (3 * (L - 1)))
    n = 3 * w * (L - 1)
    m = L * w
    tails = np.empty(n, dtype=np.int64)
    heads = np.empty(n, dtype=np.int64)
    f0 = np.empty(n)
    cost = np.empty(n)
    e = 0
    for stage in range(L - 1):
        for k in range(3):
            perm = rng.permutation(w)
            tails[e:e + w] = stage * w + np.arange(w)
            heads[e:e + w] = (stage + 1) * w + perm
            f0[e:e + w] = h[k]
            cost[e:e + w] = base * ratio ** k * (1.0 + growth) ** stage
            e += w
    u = rho * f0
    arcs = np.arange(n)
    B = sp.csr_matrix((np.concatenate([-np.ones(n), np.ones(n)]),
                       (np.concatenate([tails, heads]), np.concatenate([arcs, arcs]))),
                      shape=(m, n))
    B = _canonical(B)
    b = B @ f0
    Q = _canonical(sp.diags(-2.0 * alpha * cost / u, format="csr"))
    return dict(n=n, m=m, Q=Q, A=B, c=cost, xl=np.zeros(n), xu=u, rl=b.copy(), ru=b.copy(),
                x0=f0, seed=seed, layers=L, width=w, alpha=alpha)


def tiny_qp(n, m_e, m_i, seed, density=0.6, neg_shift=1.0, box=(0.0, 1.0)):
    """Small dense-ish instance for brute-force checks (n <= 8).

    Q symmetric with entries N(0,1) and diagonal shifted by ``-neg_shift``
    (usually indefinite); A rows drawn with the given density, equality rows
    first, then ``>=`` rows; feasible by construction through a point in the
    box interior.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 99]))
    G = rng.standard_normal((n, n))
    Qd = 0.5 * (G + G.T) - neg_shift * np.eye(n)
    m = m_e + m_i
    Ad = rng.standard_normal((m, n)) * (rng.uniform(size=(m, n)) < density)
    for j in range(m):
        if not Ad[j].any():
            Ad[j, rng.integers(n)] = 1.0
    lo, hi = box
    x_in = rng.uniform(lo + 0.2 * (hi - lo), hi - 0.2 * (hi - lo), size=n)
    ax = Ad @ x_in
    rl = np.empty(m)
    ru = np.empty(m)
    rl[:m_e] = ax[:m_e]
    ru[:m_e] = ax[:m_e]
    rl[m_e:] = ax[m_e:] - rng.uniform(0.0, 0.5, size=m_i)
    ru[m_e:] = np.inf
    c = rng.standard_normal(n)
    return dict(n=n, m=m, Q=_canonical(sp.csr_matrix(Qd)),
                A=_canonical(sp.csr_matrix(Ad)) if m else _canonical(sp.csr_matrix((0, n))),
                c=c, xl=np.full(n, lo), xu=np.full(n, hi), rl=rl, ru=ru,
                x_gen=x_in, seed=seed, instance=None)


def tiny_general_qp(n, seed, kinds=("eq", "upper", "two")):
    """Small instance (n <= 5) with one row of each requested kind:
    ``"eq"`` (rl == ru), ``"lower"`` (only rl finite), ``"upper"`` (only ru
    finite) or ``"two"`` (both finite, rl < ru).  Q, c and the box are drawn
    as in :func:`tiny_qp`; every row holds at an interior point of the box.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 98]))
    G = rng.standard_normal((n, n))
    Qd = 0.5 * (G + G.T) - np.eye(n)
    m = len(kinds)
    Ad = rng.standard_normal((m, n))
    x_in = rng.uniform(0.2, 0.8, size=n)
    ax = Ad @ x_in
    rl = np.full(m, -np.inf)
    ru = np.full(m, np.inf)
    for j, kind in enumerate(kinds):
        lo_gap, hi_gap = rng.uniform(0.0, 0.5, size=2)
        if kind == "eq":
            rl[j] = ru[j] = ax[j]
        elif kind == "lower":
            rl[j] = ax[j] - lo_gap
        elif kind == "upper":
            ru[j] = ax[j] + hi_gap
        elif kind == "two":
            rl[j] = ax[j] - lo_gap
            ru[j] = ax[j] + hi_gap
        else:
            raise ValueError(kind)
    c = rng.standard_normal(n)
    return dict(n=n, m=m, Q=_canonical(sp.csr_matrix(Qd)), A=_canonical(sp.csr_matrix(Ad)),
                c=c, xl=np.zeros(n), xu=np.ones(n), rl=rl, ru=ru, x_gen=x_in, seed=seed,
                instance=None)
