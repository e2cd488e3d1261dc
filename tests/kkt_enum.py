"""Brute-force references used to pin the oracle (test code; shares nothing
with the oracle or the library).

* ``prox_alm_minimiser``: the unique minimiser of the proximal ALM
  subproblem (paper, eq. (base-proximal-alm) with the row-wise penalties of
  Section 3.2) by enumerating which box bounds are active and solving the
  reduced linear system of each active set.
* ``kkt_points``: every KKT point of a tiny QP (problem (qp) with
  stationarity (kkt-stationarity), lambda_I <= 0 and complementarity) by
  enumerating bound activity of x and activity of the inequality rows.
* ``kkt_points_general``: the same for rows rl <= A x <= ru given on the
  caller's rows (upper-bound and two-sided rows included), enumerating each
  row's activity at its lower or upper bound.
"""

import itertools

import numpy as np


def prox_alm_minimiser(Q, c, AE, bE, AI, bI, xl, xu, z, lamE, lamI, sigE, sigI, gamma):
    """min over xl <= x <= xu, s >= bI of
       1/2 x'Qx + c'x + lamE'(AE x - bE) + 1/2 sum sigE (AE x - bE)^2
       + lamI'(AI x - s) + 1/2 sum sigI (AI x - s)^2 + ||x - z||^2 / (2 gamma).
    Returns (x, s)."""
    n = Q.shape[0]
    mi = AI.shape[0]
    SE = np.diag(sigE)
    SI = np.diag(sigI)
    Hxx = Q + np.eye(n) / gamma + AE.T @ SE @ AE + AI.T @ SI @ AI
    Hxs = -AI.T @ SI
    Hss = SI
    H = np.block([[Hxx, Hxs], [Hxs.T, Hss]]) if mi else Hxx
    g = np.concatenate([c - z / gamma + AE.T @ (lamE - SE @ bE) + AI.T @ lamI, -lamI])
    lo = np.concatenate([xl, bI])
    hi = np.concatenate([xu, np.full(mi, np.inf)])
    d = n + mi
    choices = [(-1, 0, 1)] * n + [(-1, 0)] * mi
    best = None
    for act in itertools.product(*choices):
        act = np.array(act)
        u = np.zeros(d)
        fixed = act != 0
        u[act == -1] = lo[act == -1]
        u[act == 1] = hi[act == 1]
        if not np.all(np.isfinite(u[fixed])):
            continue
        free = ~fixed
        if free.any():
            rhs = -(g[free] + H[np.ix_(free, fixed)] @ u[fixed])
            u[free] = np.linalg.solve(H[np.ix_(free, free)], rhs)
        grad = H @ u + g
        tol = 1e-9 * (1 + np.abs(g).max())
        if np.any(u < lo - tol) or np.any(u > hi + tol):
            continue
        if np.any(grad[act == -1] < -tol) or np.any(grad[act == 1] > tol):
            continue
        best = u
        break
    assert best is not None, "no active set satisfied the optimality conditions"
    return best[:n], best[n:]


def kkt_points(Q, c, AE, bE, AI, bI, xl, xu, tol=1e-9):
    """All KKT points (x, lamE, lamI) of the tiny QP."""
    n = Q.shape[0]
    me, mi = AE.shape[0], AI.shape[0]
    out = []
    for xa in itertools.product((-1, 0, 1), repeat=n):
        xa = np.array(xa)
        xfix = np.where(xa == -1, xl, np.where(xa == 1, xu, np.nan))
        if np.any(~np.isfinite(xfix[xa != 0])):
            continue
        for ia in itertools.product((0, 1), repeat=mi):
            ia = np.array(ia, dtype=bool)
            free = np.nonzero(xa == 0)[0]
            nf = free.size
            AIa = AI[ia]
            rows = []
            rhs = []
            # stationarity on free components: Q_f x + c_f + AE_f' lamE + AIa_f' lamIa = 0
            na = AIa.shape[0]
            nv = nf + me + na
            for i in free:
                row = np.zeros(nv)
                row[:nf] = Q[i, free]
                row[nf:nf + me] = AE[:, i]
                row[nf + me:] = AIa[:, i]
                rows.append(row)
                rhs.append(-(c[i] + Q[i, xa != 0] @ xfix[xa != 0]))
            for j in range(me):
                row = np.zeros(nv)
                row[:nf] = AE[j, free]
                rows.append(row)
                rhs.append(bE[j] - AE[j, xa != 0] @ xfix[xa != 0])
            for j in np.nonzero(ia)[0]:
                row = np.zeros(nv)
                row[:nf] = AI[j, free]
                rows.append(row)
                rhs.append(bI[j] - AI[j, xa != 0] @ xfix[xa != 0])
            if nv == 0:
                sol = np.zeros(0)
            else:
                M = np.array(rows).reshape(-1, nv)
                b = np.array(rhs)
                if M.shape[0] != nv or abs(np.linalg.det(M)) < 1e-12:
                    continue
                sol = np.linalg.solve(M, b)
            x = xfix.copy()
            x[free] = sol[:nf]
            lamE = sol[nf:nf + me]
            lamI = np.zeros(mi)
            lamI[ia] = sol[nf + me:]
            if np.any(x < xl - tol) or np.any(x > xu + tol):
                continue
            if np.any(AE @ x - bE > tol) or np.any(AE @ x - bE < -tol):
                continue
            if np.any(AI @ x < bI - tol):
                continue
            if np.any(lamI > tol):
                continue
            g = Q @ x + c + AE.T @ lamE + AI.T @ lamI
            if np.any(g[xa == -1] < -tol) or np.any(g[xa == 1] > tol):
                continue
            out.append((x, lamE, lamI))
    return out


def kkt_points_general(Q, c, A, rl, ru, xl, xu, tol=1e-9):
    """All KKT points (x, lam) of a tiny QP with general rows
    rl <= A x <= ru (rl == ru an equality), in the sign convention
    Qx + c + A'lam + N_[xl,xu](x) contains 0: lam_j <= 0 when row j sits at
    its lower bound, >= 0 at its upper bound, free on an equality row, 0 on
    an inactive row.  Enumerates bound activity of every variable and every
    row directly on the caller's rows (no conversion to another form)."""
    n = Q.shape[0]
    m = A.shape[0]
    out = []
    row_states = []
    for j in range(m):
        if rl[j] == ru[j]:
            row_states.append((2,))          # equality: always active
        else:
            st = [0]
            if np.isfinite(rl[j]):
                st.append(-1)
            if np.isfinite(ru[j]):
                st.append(1)
            row_states.append(tuple(st))
    for xa in itertools.product((-1, 0, 1), repeat=n):
        xa = np.array(xa)
        xfix = np.where(xa == -1, xl, np.where(xa == 1, xu, np.nan))
        if np.any(~np.isfinite(xfix[xa != 0])):
            continue
        for ra in itertools.product(*row_states):
            ra = np.array(ra, dtype=int)
            act = np.nonzero(ra != 0)[0]
            target = np.array([rl[j] if ra[j] in (-1, 2) else ru[j] for j in act])
            free = np.nonzero(xa == 0)[0]
            nf, na = free.size, act.size
            nv = nf + na
            M = np.zeros((nf + na, nv))
            rhs = np.zeros(nf + na)
            fixed = xa != 0
            for r, i in enumerate(free):
                M[r, :nf] = Q[i, free]
                M[r, nf:] = A[act, i]
                rhs[r] = -(c[i] + Q[i, fixed] @ xfix[fixed])
            for r, j in enumerate(act):
                M[nf + r, :nf] = A[j, free]
                rhs[nf + r] = target[r] - A[j, fixed] @ xfix[fixed]
            if nv:
                if abs(np.linalg.det(M)) < 1e-12:
                    continue
                sol = np.linalg.solve(M, rhs)
            else:
                sol = np.zeros(0)
            x = xfix.copy()
            x[free] = sol[:nf]
            lam = np.zeros(m)
            lam[act] = sol[nf:]
            if np.any(x < xl - tol) or np.any(x > xu + tol):
                continue
            ax = A @ x
            if np.any(ax < rl - tol) or np.any(ax > ru + tol):
                continue
            if np.any((ra == -1) & (lam > tol)) or np.any((ra == 1) & (lam < -tol)):
                continue
            g = Q @ x + c + A.T @ lam
            if np.any(g[xa == -1] < -tol) or np.any(g[xa == 1] > tol):
                continue
            out.append((x, lam))
    return out
