"""Pins of the FP64 CPU oracle against what the paper and the mathematics
fix, independent of the oracle's own code paths:

* brute-force active-set minimiser of the proximal ALM subproblem
  (eq. (base-proximal-alm), row-wise penalties): the residual-form inner QP
  (eq. (inner-qp)) solved by the oracle's PDHG must reach it;
* PDHG fixed point = KKT point: one trial step (pdqp-trial) from the
  minimiser and its multiplier returns the same point with zero acceptance
  sums and zero inner residuals;
* the residual-form objective equals the proximal ALM objective minus the
  omitted constant ||z||^2 / (2 gamma) on the affine set Bw = h;
* after an exact inner solve the multiplier update gives lambda = -y;
* the full method returns one of the brute-force-enumerated KKT points of
  tiny nonconvex QPs;
* closed forms (m = 0, diagonal Q), Ruiz equilibration limits, Lanczos
  against a dense eigensolver, the step-size row identity, the averaging
  weights, the acceptance test's exact thresholds on 1-D examples;
* mutation checks: plausible mistakes planted in the oracle make the pins
  fail.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from oracle import pdnqp_oracle as O
from tests.kkt_enum import kkt_points, prox_alm_minimiser


def _unit_scaled(p):
    """The normalised problem with unit outer scaling and c_obj = 1."""
    P = O.normalise(p)
    return O.Scaled(n=P.n, m_e=P.m_e, m_i=P.m_i, Q=P.Q, c=P.c, A=P.A, b=P.b, xl=P.xl,
                    xu=P.xu, Dc=np.ones(P.m_e + P.m_i), Dx=np.ones(P.n), c_obj=1.0)


def _inner_case(seed, n=4, m_e=1, m_i=2):
    p = qpgen.tiny_qp(n, m_e, m_i, seed)
    S = _unit_scaled(p)
    rng = np.random.default_rng(seed + 1000)
    st = O.Settings()
    gamma, _ = O.choose_gamma(S.Q, st)
    m = S.m_e + S.m_i
    z = rng.uniform(0, 1, S.n)
    lam = np.concatenate([rng.normal(size=S.m_e), -np.abs(rng.normal(size=S.m_i))])
    sigma = rng.uniform(0.5, 5.0, m)
    x0 = rng.uniform(0, 1, S.n)
    return p, S, gamma, z, lam, sigma, x0


def _solve_inner_tight(S, gamma, z, lam, sigma, x0, st=None):
    st = st or O.Settings(max_inner=400000)
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    si = O.scale_inner(qp, sigma, st)
    w0 = O.warm_start(S, x0, lam, sigma)
    state = O.new_inner_state(qp, si, w0, -lam, 1.0, st)
    status, _ = O.inner_solve(state, 1.0, 1e-12, 1e-12, st, O.Counters())
    return status, qp, si, state


def _brute(S, gamma, z, lam, sigma):
    me = S.m_e
    Qd = S.Q.toarray()
    Ad = S.A.toarray()
    return prox_alm_minimiser(Qd, S.c, Ad[:me], S.b[:me], Ad[me:], S.b[me:], S.xl, S.xu, z,
                              lam[:me], lam[me:], sigma[:me], sigma[me:], gamma)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_inner_solve_reaches_bruteforce_minimiser(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    status, qp, si, state = _solve_inner_tight(S, gamma, z, lam, sigma, x0)
    assert status == O.INNER_CONVERGED
    w = si.Sw * state.w
    n, mi = S.n, S.m_i
    xb, sb = _brute(S, gamma, z, lam, sigma)
    np.testing.assert_allclose(w[:n], xb, atol=1e-7)
    np.testing.assert_allclose(w[n:n + mi], sb, atol=1e-7)
    # residual blocks equal their definitions at the solution
    ax = S.A @ w[:n]
    r = w[n + mi:]
    np.testing.assert_allclose(r[:S.m_e], ax[:S.m_e] - S.b[:S.m_e], atol=1e-7)
    np.testing.assert_allclose(r[S.m_e:], ax[S.m_e:] - w[n:n + mi], atol=1e-7)


def _kkt_point(S, gamma, z, lam, sigma):
    xb, sb = _brute(S, gamma, z, lam, sigma)
    me = S.m_e
    ax = S.A @ xb
    r = np.concatenate([ax[:me] - S.b[:me], ax[me:] - sb])
    w = np.concatenate([xb, sb, r])
    y = -(sigma * r + lam)          # r-block stationarity: sigma r + lambda + y = 0
    return w, y


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_pdhg_fixed_point_is_kkt_point(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    st = O.Settings()
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    si = O.scale_inner(qp, sigma, st)
    w, y = _kkt_point(S, gamma, z, lam, sigma)
    rp, rd, _, _ = O.inner_residuals(qp, w, y)
    assert rp < 1e-10 and rd < 1e-9
    wh, yh = w / si.Sw, y / si.Ey
    for omega in (0.3, 1.0, 7.0):
        tau, eta = O.diagonal_steps(si.m_w, si.m_y, omega, st)
        for alpha, beta in ((1.0, 0.0), (0.4, 0.7)):
            w_tr, y_tr = O.trial_step(si, wh, wh, yh, tau, eta, alpha, beta)
            np.testing.assert_allclose(w_tr, wh, atol=1e-9 * (1 + np.abs(wh).max()))
            np.testing.assert_allclose(y_tr, yh, atol=1e-9 * (1 + np.abs(yh).max()))
            lhs, rhs = O.adaptive_condition(si, w_tr - wh, y_tr - yh, tau, eta)
            assert lhs < 1e-15 and rhs < 1e-15


@pytest.mark.parametrize("seed", [1, 7])
def test_residual_form_equals_prox_alm_objective(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    rng = np.random.default_rng(seed)
    me = S.m_e
    for _ in range(5):
        x = rng.uniform(0, 1, S.n)
        s = S.b[me:] + rng.uniform(0, 1, S.m_i)
        ax = S.A @ x
        r = np.concatenate([ax[:me] - S.b[:me], ax[me:] - s])
        w = np.concatenate([x, s, r])
        np.testing.assert_allclose(qp.B @ w, qp.h, atol=1e-12)
        inner = 0.5 * w @ (qp.H @ w) + qp.q @ w
        # augmented Lagrangian (base-alm) with row-wise penalties + proximal term
        Qd = S.Q.toarray()
        rE = ax[:me] - S.b[:me]
        rI = ax[me:] - s
        alm = (0.5 * x @ Qd @ x + S.c @ x + lam[:me] @ rE + 0.5 * np.sum(sigma[:me] * rE ** 2)
               + lam[me:] @ rI + 0.5 * np.sum(sigma[me:] * rI ** 2))
        prox = alm + np.sum((x - z) ** 2) / (2 * gamma)
        assert inner == pytest.approx(prox - np.sum(z ** 2) / (2 * gamma), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("seed", [2, 3])
def test_warm_start_restores_residual_definitions(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    w0 = O.warm_start(S, x0, lam, sigma)
    np.testing.assert_allclose(qp.B @ w0, qp.h, atol=1e-13)
    s0 = w0[S.n:S.n + S.m_i]
    assert np.all(s0 >= S.b[S.m_e:])


@pytest.mark.parametrize("seed", [1, 4])
def test_multiplier_update_equals_minus_inner_dual(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    status, qp, si, state = _solve_inner_tight(S, gamma, z, lam, sigma, x0)
    assert status == O.INNER_CONVERGED
    w = si.Sw * state.w
    y = si.Ey * state.y
    _, s_new, lam_new = O.multiplier_update(S, w[:S.n], lam, sigma)
    np.testing.assert_allclose(lam_new, -y, atol=1e-6)
    np.testing.assert_allclose(s_new, w[S.n:S.n + S.m_i], atol=1e-7)
    assert np.all(lam_new[S.m_e:] <= 0)


def _kkt_residual(p, x, lam):
    """Independent stationarity/feasibility measure of the original QP."""
    Q = p["Q"].toarray()
    A = p["A"].toarray()
    g = Q @ x + p["c"] + A.T @ lam
    proj = np.clip(x - g, p["xl"], p["xu"])
    ax = A @ x
    feas = np.maximum(np.maximum(p["rl"] - ax, ax - p["ru"]), 0)
    return max(np.abs(x - proj).max(), feas.max() if feas.size else 0.0)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mode", [O.SCALE_RUIZ_A, O.SCALE_RUIZ_QA])
def test_full_method_returns_enumerated_kkt_point(seed, mode):
    p = qpgen.tiny_qp(3, 1, 1, seed)
    st = O.Settings(eps_abs=1e-9, eps_rel=1e-9, max_outer=20000, outer_scaling=mode)
    res = O.solve(p, st)
    assert res.status == O.SOLVED
    assert _kkt_residual(p, res.x, res.lam) < 1e-6
    Q = p["Q"].toarray()
    A = p["A"].toarray()
    pts = kkt_points(Q, p["c"], A[:1], p["rl"][:1], A[1:], p["rl"][1:], p["xl"], p["xu"])
    assert pts, "enumeration found no KKT point"
    dist = min(np.abs(res.x - x).max() for x, _, _ in pts)
    assert dist < 1e-5
    # lambda_I <= 0 on the inequality row, multiplier close to the KKT one
    assert res.lam[1] <= 1e-9
    best = min(pts, key=lambda t: np.abs(res.x - t[0]).max())
    np.testing.assert_allclose(res.lam, np.concatenate([best[1], best[2]]), atol=1e-4)


def test_unconstrained_diagonal_convex_closed_form():
    rng = np.random.default_rng(3)
    n = 7
    d = rng.uniform(0.5, 3.0, n)
    c = rng.normal(size=n) * 2
    p = dict(Q=sp.diags(d, format="csr"), A=sp.csr_matrix((0, n)), c=c, xl=np.zeros(n),
             xu=np.ones(n), rl=np.zeros(0), ru=np.zeros(0))
    res = O.solve(p, O.Settings(eps_abs=1e-10, eps_rel=1e-10))
    assert res.status == O.SOLVED
    np.testing.assert_allclose(res.x, np.clip(-c / d, 0, 1), atol=1e-8)


def test_inner_minimiser_without_constraints_closed_form():
    rng = np.random.default_rng(5)
    n = 6
    d = rng.uniform(-2.0, 3.0, n)
    c = rng.normal(size=n)
    p = dict(Q=sp.diags(d, format="csr"), A=sp.csr_matrix((0, n)), c=c, xl=np.zeros(n),
             xu=np.ones(n), rl=np.zeros(0), ru=np.zeros(0))
    S = _unit_scaled(p)
    gamma, _ = O.choose_gamma(S.Q, O.Settings())
    assert np.all(d + 1 / gamma > 0)
    z = rng.uniform(0, 1, n)
    status, qp, si, state = _solve_inner_tight(S, gamma, z, np.zeros(0), np.zeros(0),
                                               np.zeros(n))
    assert status == O.INNER_CONVERGED
    np.testing.assert_allclose(si.Sw * state.w, np.clip((z / gamma - c) / (d + 1 / gamma), 0, 1),
                               atol=1e-9)


def test_ruiz_equilibrates_rows_and_columns():
    rng = np.random.default_rng(0)
    M = sp.random(40, 60, density=0.15, random_state=1, format="csr")
    M.data = rng.normal(size=M.nnz) * 10 ** rng.uniform(-3, 3, M.nnz)
    M = M + sp.eye(40, 60)          # no empty rows or columns
    dr, dc = O.ruiz(M, 60)
    S = abs(sp.diags(dr) @ M @ sp.diags(dc))
    np.testing.assert_allclose(S.max(axis=1).toarray().ravel(), 1.0, atol=1e-6)
    np.testing.assert_allclose(S.max(axis=0).toarray().ravel(), 1.0, atol=1e-6)
    dr2, dc2 = O.ruiz(M.T, 60)
    np.testing.assert_allclose(dr2, dc, rtol=1e-12)
    np.testing.assert_allclose(dc2, dr, rtol=1e-12)


def test_lanczos_matches_dense_eigensolver():
    rng = np.random.default_rng(2)
    G = rng.normal(size=(30, 30))
    Q = sp.csr_matrix(G + G.T)
    lam = O.lanczos_min_eig(Q, 30)
    assert lam == pytest.approx(np.linalg.eigvalsh(G + G.T)[0], rel=1e-8)


def test_gamma_makes_scaled_hessian_positive_definite():
    p = qpgen.workload("small", 1)
    for mode in (O.SCALE_RUIZ_A, O.SCALE_RUIZ_QA):
        P = O.normalise(p)
        S = O.outer_scale(P, np.zeros(P.n), 8, mode)
        gamma, lam_hat = O.choose_gamma(S.Q, O.Settings())
        ev = np.linalg.eigvalsh(S.Q.toarray())
        assert lam_hat >= ev[0] - 1e-8          # a Ritz value never undershoots
        assert ev[0] + 1 / gamma > 0


@pytest.mark.parametrize("seed", [1, 3])
def test_diagonal_steps_row_identity(seed):
    """With tau = 0.99/(omega m_w) and eta = 0.99 omega / m_y, every row of
    eta^(1/2) B tau^(1/2) has squared norm 0.99^2."""
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    st = O.Settings()
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    si = O.scale_inner(qp, sigma, st)
    tau, eta = O.diagonal_steps(si.m_w, si.m_y, 2.5, st)
    rows = np.asarray(si.B.multiply(si.B) @ tau).ravel() * eta
    np.testing.assert_allclose(rows, 0.99 ** 2, rtol=1e-12)
    assert np.all(si.m_w > 0)


def test_averages_weight_iterates_linearly():
    """alpha_N = 2/(N+2) makes the average after N accepted steps the
    mean of w_1..w_N with weights 1..N."""
    p, S, gamma, z, lam, sigma, x0 = _inner_case(3)
    st = O.Settings(check_every=10 ** 9, max_inner=7, restart_suff=0.0, restart_nec=0.0,
                    restart_art=10.0)
    qp = O.form_inner_qp(S, z, lam, sigma, gamma)
    si = O.scale_inner(qp, sigma, st)
    state = O.new_inner_state(qp, si, O.warm_start(S, x0, lam, sigma), -lam, 1.0, st)
    tr = O.Trace(max_iters=100)
    status, _ = O.inner_solve(state, 1.0, 0.0, 0.0, st, O.Counters(), tr)
    assert status == O.INNER_ITER_LIMIT and len(tr.w) == 7
    wts = np.arange(1, 8, dtype=float)
    avg = (wts[:, None] * np.array(tr.w)).sum(0) / wts.sum()
    np.testing.assert_allclose(si.Sw * state.wbar, avg, rtol=1e-12, atol=1e-13)


def _one_dim(h_val, b_val=None):
    H = sp.csr_matrix(np.array([[h_val]]))
    if b_val is None:
        B = sp.csr_matrix((0, 1))
        h = np.zeros(0)
    else:
        B = sp.csr_matrix(np.array([[b_val]]))
        h = np.array([0.7])
    return O.ScaledInner(H=H, q=np.array([1.3]), B=B, h=h, lo=np.array([-np.inf]),
                         hi=np.array([np.inf]), Sw=np.ones(1), Ey=np.ones(B.shape[0]),
                         m_w=np.ones(1), m_y=np.ones(B.shape[0]))


def test_acceptance_threshold_quadratic_term():
    """m = 0, one variable: the trial is accepted exactly when tau*H <= 1."""
    si = _one_dim(4.0)
    w = np.array([0.2])
    for tau_v, expect in ((0.24, True), (0.25, True), (0.26, False), (1.0, False)):
        tau = np.array([tau_v])
        w_tr, y_tr = O.trial_step(si, w, w, np.zeros(0), tau, np.zeros(0), 1.0, 0.0)
        lhs, rhs = O.adaptive_condition(si, w_tr - w, y_tr, tau, np.zeros(0))
        assert (lhs >= rhs) == expect


def test_acceptance_threshold_coupling_term():
    """H = 0, one variable, one row b: accepted whenever tau*eta*b^2 <= 1
    (AM-GM); rejected when the step sizes are balanced with tau*eta*b^2 = 4."""
    si = _one_dim(0.0, b_val=2.0)
    rng = np.random.default_rng(0)
    for _ in range(50):
        tau = np.array([rng.uniform(0.01, 1.0)])
        eta = np.array([rng.uniform(0.0, 1.0) / (4 * tau[0])])
        w = rng.normal(size=1)
        y = rng.normal(size=1)
        w_tr, y_tr = O.trial_step(si, w, w, y, tau, eta, 1.0, 0.0)
        lhs, rhs = O.adaptive_condition(si, w_tr - w, y_tr - y, tau, eta)
        assert lhs >= rhs
    # tau*eta*b^2 = 4 with |dw|/sqrt(tau) == |dy|/sqrt(eta): lhs = dw^2/tau, rhs = 2 dw^2/tau
    tau = np.array([1.0])
    eta = np.array([1.0])
    dw, dy = np.array([0.5]), np.array([0.5])
    lhs, rhs = O.adaptive_condition(si, dw, dy, tau, eta)
    assert lhs < rhs


# --------------------------------------------------------------------------
# Mutation checks: plant a plausible mistake in the oracle and require that
# a pin above catches it.
# --------------------------------------------------------------------------

def _inner_matches_bruteforce(seed):
    p, S, gamma, z, lam, sigma, x0 = _inner_case(seed)
    st = O.Settings(max_inner=30000)
    try:
        status, qp, si, state = _solve_inner_tight(S, gamma, z, lam, sigma, x0, st)
    except (FloatingPointError, ValueError, OverflowError):
        return False
    if status != O.INNER_CONVERGED:
        return False
    w = si.Sw * state.w
    xb, sb = _brute(S, gamma, z, lam, sigma)
    return bool(np.abs(w[:S.n] - xb).max() < 1e-6)


def test_mutation_dual_sign_in_primal_step(monkeypatch):
    def bad_trial(si, w, wbar, y, tau, eta, alpha, beta):
        grad = si.q + (1 - alpha) * (si.H @ wbar) + alpha * (si.H @ w) + si.B.T @ y
        w_tr = np.clip(w - tau * grad, si.lo, si.hi)
        Bw_tr = si.B @ w_tr
        return w_tr, y + eta * (si.h - Bw_tr - beta * (Bw_tr - si.B @ w))
    assert _inner_matches_bruteforce(1)
    monkeypatch.setattr(O, "trial_step", bad_trial)
    assert not _inner_matches_bruteforce(1)


def test_mutation_proximal_centre_sign(monkeypatch):
    orig = O.form_inner_qp

    def bad_form(S, z, lam, sigma, gamma):
        qp = orig(S, z, lam, sigma, gamma)
        qp.q[:S.n] = S.c + z / gamma
        return qp
    monkeypatch.setattr(O, "form_inner_qp", bad_form)
    assert not _inner_matches_bruteforce(2)


def test_mutation_penalty_block_dropped(monkeypatch):
    orig = O.form_inner_qp

    def bad_form(S, z, lam, sigma, gamma):
        qp = orig(S, z, lam, sigma, gamma)
        n, mi = S.n, S.m_i
        d = qp.H.diagonal()
        d[n + mi:] = 0.0
        qp.H = sp.csr_matrix(sp.block_diag([qp.H[:n, :n], sp.diags(d[n:])]))
        return qp
    monkeypatch.setattr(O, "form_inner_qp", bad_form)
    assert not _inner_matches_bruteforce(3)


# ---------------------------------------------------------------------------
# Anderson acceleration (Section 3.2, "Anderson acceleration")
# ---------------------------------------------------------------------------

def test_anderson_single_point_is_plain_iteration():
    g = np.array([1.0, -2.0, 3.0])
    assert np.array_equal(O.anderson_step([np.zeros(3)], [g], 0.0), g)


def test_anderson_matches_constrained_form():
    """The difference form equals the classical constrained form of Type-II
    Anderson mixing: alpha = argmin ||sum_j alpha_j f_j||_2 subject to
    sum_j alpha_j = 1, next point = sum_j alpha_j G_j."""
    rng = np.random.default_rng(21)
    U = [rng.normal(size=7) for _ in range(4)]
    G = [rng.normal(size=7) for _ in range(4)]
    v1 = O.anderson_step(U, G, 0.0)
    F = np.column_stack([G[j] - U[j] for j in range(4)])
    K = np.zeros((5, 5))
    K[:4, :4] = 2.0 * F.T @ F
    K[:4, 4] = 1.0
    K[4, :4] = 1.0
    rhs = np.zeros(5)
    rhs[4] = 1.0
    alpha = np.linalg.solve(K, rhs)[:4]
    v2 = sum(alpha[j] * G[j] for j in range(4))
    np.testing.assert_allclose(v1, v2, rtol=1e-10, atol=1e-12)


def test_anderson_affine_map_finite_termination():
    """On an affine contraction u -> M u + b in R^d, Type-II Anderson with
    memory >= d reaches the fixed point (I - M)^{-1} b after d + 1 map
    evaluations: its iterates are those of GMRES on (I - M) u = b, which
    terminates in at most d steps."""
    rng = np.random.default_rng(5)
    d = 4
    M = rng.normal(size=(d, d))
    M *= 0.5 / np.abs(np.linalg.eigvals(M)).max()
    b = rng.normal(size=d)
    ustar = np.linalg.solve(np.eye(d) - M, b)
    U, G = [], []
    u = np.zeros(d)
    for _ in range(d + 1):
        U.append(u)
        G.append(M @ u + b)
        u = O.anderson_step(U, G, 0.0)
    assert np.abs(u - ustar).max() <= 1e-9 * max(1.0, np.abs(ustar).max())
    # the plain iteration is still far away after as many steps
    v = np.zeros(d)
    for _ in range(d + 1):
        v = M @ v + b
    assert np.abs(v - ustar).max() > 1e-3


def test_anderson_in_solve_keeps_termination():
    """With the paper's memory m_A = 5 the method still ends at a point that
    meets the outer test, and the extrapolation is actually used."""
    prob = qpgen.random_indefinite_qp(300, 150, 5, 4, 3, instance=1)
    st = O.Settings(anderson_mem=5, outer_scaling=2, max_outer=3000)
    res = O.solve(prob, st)
    assert res.status == O.SOLVED
    assert O.passes_external(res, 1e-3, 1e-3)
    assert res.anderson_steps > 0
