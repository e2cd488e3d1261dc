"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Iterate parity: after every accepted inner iteration of the first 1000 the
unscaled inner iterate (w, y) must satisfy
    ||w_gpu - w_oracle||_inf <= 1e-9 * max(1, ||w_oracle||_inf)
(same for y), and the accept/reject and check decision sequences must be
identical.  Full solves: same status, and the returned point matches the
oracle's.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from oracle import pdnqp_oracle as O

pytestmark = pytest.mark.gpu

PARITY_TOL = 1e-9


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    P.load()
    return P


def _oracle_settings(**kw):
    return O.Settings(**kw)


def _gpu_kwargs(st: O.Settings):
    """Same parameter values for the library."""
    keys = ["max_inner", "ruiz_sweeps", "sigma_init", "theta_sigma", "delta_gamma", "rho_in_min",
            "rho_in_max", "rho_z", "check_every", "max_rejects", "restart_suff", "restart_nec",
            "restart_art", "shrink_safety", "shrink_min", "shrink_max", "omega0", "sigma_growth",
            "sigma_max", "sigma0_min", "sigma0_max", "lanczos_iters", "gamma_override",
            "step_boost", "outer_scaling", "anderson_mem", "anderson_reg", "delta_floor",
            "external_halvings", "delta0", "kkt_pass_limit"]
    kw = {k: getattr(st, k) for k in keys}
    kw["max_outer"] = int(min(st.max_outer, 2**62))
    kw["penalty_gate"] = int(st.penalty_gate)
    kw["center_floor"] = int(st.center_floor)
    kw["time_limit_s"] = st.time_limit if math.isfinite(st.time_limit) else math.inf
    return kw


def run_pair(P, prob, st, iters=1000, trials=4000, **lib_only):
    tr = O.Trace(max_iters=iters)
    res_o = O.solve(prob, st, trace=tr)
    s = P.Solver.from_problem(prob, trace_iters=iters, trace_trials=trials, **_gpu_kwargs(st),
                              **lib_only)
    x, lam, info = s.solve(st.eps_abs, st.eps_rel)
    t = s.trace()
    return res_o, tr, (x, lam, info), t, s


def assert_meets_tolerance(info, eps_abs, eps_rel):
    """A SOLVED result passes the KKT test on the caller's unscaled problem
    (primal residual with bound violation, projected stationarity), as the
    paper's experimental protocol requires of an accepted point."""
    assert info["r_p"] <= eps_abs + eps_rel * info["s_p"], (info["r_p"], info["s_p"])
    assert info["r_d"] <= eps_abs + eps_rel * info["s_d"], (info["r_d"], info["s_d"])


def assert_iterate_parity(tr, t, n_expect=None):
    n = min(len(tr.w), t["w"].shape[0])
    if n_expect is not None:
        assert n >= n_expect, f"only {n} accepted iterations recorded"
    assert n == len(tr.w) == t["w"].shape[0]
    W = np.array(tr.w)
    Y = np.array(tr.y) if tr.y and np.array(tr.y).size else np.zeros((n, 0))
    for k in range(n):
        wn = max(1.0, np.abs(W[k]).max())
        dw = np.abs(t["w"][k] - W[k]).max() / wn
        assert dw <= PARITY_TOL, f"w differs at accepted iteration {k}: {dw:.3e}"
        if Y.shape[1]:
            yn = max(1.0, np.abs(Y[k]).max())
            dy = np.abs(t["y"][k] - Y[k]).max() / yn
            assert dy <= PARITY_TOL, f"y differs at accepted iteration {k}: {dy:.3e}"


def assert_decision_parity(tr, t, window=None):
    """Accept/reject and check decisions agree inside the window of trials
    that produced the recorded iterates (all trials when window is None).

    Beyond the window the two runs are not expected to stay together:
    rounding-order differences (about 1e-16 per operation) are amplified by
    the method's continuous dependence on the iterate (shrink factors,
    primal weight, penalties), roughly 1e-12 after 1000 iterations and 1e-9
    after 2000 on the small workload, until a decision eventually flips."""
    nt = min(len(tr.trials), t["trials"].shape[0])
    if window is not None:
        nt = min(nt, window)
    acc_o = np.array([a for (_, _, a) in tr.trials[:nt]])
    acc_g = t["trials"][:nt, 2] > 0.5
    assert np.array_equal(acc_o, acc_g), "accept/reject sequences differ"
    lhs_o = np.array([l for (l, _, _) in tr.trials[:nt]])
    # the sums lose relative accuracy to cancellation in dw once steps are tiny
    np.testing.assert_allclose(t["trials"][:nt, 0], lhs_o, rtol=1e-5, atol=1e-300)
    nc = min(len(tr.checks), t["checks"].shape[0])
    kinds = {"continue": 0, "restart": 1, "converged": 2}
    compared = 0
    for k in range(nc):
        kind, tt, which, trials_o, ratio = tr.checks[k]
        if window is not None and trials_o > window:
            break
        g = t["checks"][k]
        assert (g[0], g[1], g[2], g[3]) == (kinds[kind], tt, which, trials_o), \
            f"check {k} differs inside the parity window: oracle {tr.checks[k]}, gpu {g.tolist()}"
        compared += 1
    return compared


def window_of(tr):
    """Number of trials up to and including the last recorded accepted one."""
    acc = 0
    for k, (_, _, a) in enumerate(tr.trials):
        acc += bool(a)
        if acc == len(tr.w):
            return k + 1
    return len(tr.trials)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("mode", [0, 2])
def test_small_first_1000_iterations(P, seed, mode):
    prob = qpgen.workload("small", seed)
    st = _oracle_settings(max_outer=40, outer_scaling=mode)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st)
    assert_iterate_parity(tr, t, n_expect=1000)
    assert_decision_parity(tr, t, window_of(tr))
    assert info["gamma"] == pytest.approx(res_o.gamma, rel=1e-10)


@pytest.mark.parametrize("seed,grid", [(1, 0), (3, 0), (1, 2), (3, 6)])
def test_two_panel_form_first_1000_iterations(P, seed, grid):
    """The two-column-panel form of the first trial product (forced here; by
    default it runs only when x exceeds one XCD's L2): same iterates and
    decisions as the oracle.  Grids of 2 and 6 workgroups make every
    workgroup of the pipelined product launches walk many row blocks."""
    prob = qpgen.workload("small", seed)
    st = _oracle_settings(max_outer=40, outer_scaling=2)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st, col_panels=2, stream_grid=grid)
    assert_iterate_parity(tr, t, n_expect=1000)
    assert_decision_parity(tr, t, window_of(tr))
    names = {k["name"] for k in s.kernel_stats()}
    assert "qa_panels" in names and "qa_rows" in names


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("mode", [0, 2])
def test_literal_rules_first_1000_iterations(P, seed, mode):
    """The paper's outer rules as stated: no penalty gate (every equality row
    and active inequality row whose residual did not fall to 0.25 of the
    previous one is raised), no floor on the centre tolerances and none on
    the inner tolerances."""
    prob = qpgen.workload("small", seed)
    st = _oracle_settings(max_outer=40, outer_scaling=mode, penalty_gate=False,
                          center_floor=False, delta_floor=0.0)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st)
    assert_iterate_parity(tr, t, n_expect=1000)
    assert_decision_parity(tr, t, window_of(tr))
    assert info["outer_iters"] >= 3


@pytest.mark.parametrize("seed", [1, 2])
def test_small_full_solve(P, seed):
    """Full solve to 1e-4: the GPU result meets the termination test, its
    reported unscaled KKT residuals are those of its point, and the first
    1000 iterations coincide with the oracle's."""
    prob = qpgen.workload("small", seed)
    st = _oracle_settings(outer_scaling=2, max_outer=5000, time_limit=120.0)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st, iters=1000, trials=100000)
    assert res_o.status == O.SOLVED
    assert info["status"] == O.SOLVED
    assert_iterate_parity(tr, t, n_expect=1000)
    assert_decision_parity(tr, t, window_of(tr))
    assert info["r_p_scaled"] <= 1e-4 + 1e-4 * info["s_p_scaled"]
    assert info["r_d_scaled"] <= 1e-4 + 1e-4 * info["s_d_scaled"]
    assert_meets_tolerance(info, 1e-4, 1e-4)
    rp, rd, sp_, sd = O.external_kkt(prob, x, lam)
    assert info["r_p"] == pytest.approx(rp, rel=1e-6, abs=1e-12)
    assert info["r_d"] == pytest.approx(rd, rel=1e-6, abs=1e-12)
    assert info["s_p"] == pytest.approx(sp_, rel=1e-12)
    assert info["s_d"] == pytest.approx(sd, rel=1e-9)
    assert np.all(x >= prob["xl"]) and np.all(x <= prob["xu"])


def _custom(n, A, rl, ru, seed, xl=None, xu=None, Qd=None):
    rng = np.random.default_rng(seed)
    if Qd is None:
        G = sp.random(n, n, density=min(1.0, 4.0 / n), random_state=seed, format="csr")
        G.data = rng.normal(size=G.nnz)
        Qd = sp.csr_matrix(G + G.T + sp.diags(rng.normal(-1, 1, n)))
    return dict(Q=sp.csr_matrix(Qd), A=sp.csr_matrix(A), c=rng.normal(size=n),
                xl=np.zeros(n) if xl is None else xl, xu=np.ones(n) if xu is None else xu,
                rl=np.asarray(rl, float), ru=np.asarray(ru, float))


def _edge_cases():
    rng = np.random.default_rng(11)
    cases = {}
    n = 37
    cases["no_rows"] = _custom(n, sp.csr_matrix((0, n)), [], [], 1)
    A = sp.random(20, n, density=0.1, random_state=2, format="csr")
    A.data = rng.normal(size=A.nnz)
    x0 = rng.uniform(0.2, 0.8, n)
    ax = A @ x0
    cases["equalities_only"] = _custom(n, A, ax, ax, 3)
    cases["inequalities_only"] = _custom(n, A, ax - 0.3, np.full(20, np.inf), 4)
    ru = ax + 0.2
    cases["upper_rows_negated"] = _custom(n, A, np.full(20, -np.inf), ru, 5)
    rl2 = ax - 0.1
    ru2 = ax + 0.1
    rl2[::3] = ax[::3]
    ru2[::3] = ax[::3]
    cases["two_sided_rows"] = _custom(n, A, rl2, ru2, 6)
    A2 = A.tolil()
    A2[5, :] = 0
    A2 = sp.csr_matrix(A2)
    A2.eliminate_zeros()
    cases["empty_row_and_free_vars"] = _custom(
        n, A2, A2 @ x0 - 0.05, np.full(20, np.inf), 7,
        xl=np.where(np.arange(n) % 4 == 0, -np.inf, 0.0),
        xu=np.where(np.arange(n) % 4 == 0, np.inf, 1.0),
        Qd=sp.diags(rng.uniform(0.5, 2.0, n)))
    cases["single_variable"] = _custom(1, sp.csr_matrix(np.array([[2.0]])), [0.5], [np.inf], 8,
                                       Qd=sp.csr_matrix(np.array([[-1.0]])))
    nr = 1037
    Ar = sp.random(517, nr, density=0.006, random_state=9, format="csr")
    Ar.data = rng.normal(size=Ar.nnz)
    cases["ragged_tail_rows"] = _custom(nr, Ar, Ar @ np.full(nr, 0.5) - 0.2,
                                        np.full(517, np.inf), 9)
    # a row longer than any stream tile (4500 nonzeros), next to short rows
    nd = 4500
    Ad = sp.vstack([sp.csr_matrix(rng.normal(size=(1, nd))),
                    sp.random(3, nd, density=3.0 / nd, random_state=10, format="csr")]).tocsr()
    xd = rng.uniform(0.2, 0.8, nd)
    axd = Ad @ xd
    cases["row_longer_than_tile"] = _custom(
        nd, Ad, np.concatenate([axd[:1], axd[1:] - 0.1]),
        np.concatenate([axd[:1], np.full(3, np.inf)]), 12,
        Qd=sp.diags(rng.uniform(0.5, 2.0, nd)).tocsr())
    return cases


EDGE = _edge_cases()


@pytest.mark.parametrize("grid", [0, 2])
@pytest.mark.parametrize("panels", [1, 2])
@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases_iterate_parity(P, name, panels, grid):
    """Edge cases in both forms of the first product; with a grid of 2
    workgroups per pipelined launch each workgroup walks all of its row
    blocks in turn (empty blocks, a row longer than a tile between short
    rows, a ragged last block)."""
    prob = EDGE[name]
    st = _oracle_settings(max_outer=12, outer_scaling=2)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st, iters=400, trials=800,
                                               col_panels=panels, stream_grid=grid)
    assert_iterate_parity(tr, t)
    assert_decision_parity(tr, t, window_of(tr))
    assert info["status"] == res_o.status
    np.testing.assert_allclose(x, res_o.x, atol=1e-8 * max(1, np.abs(res_o.x).max()))


def test_rejection_limit_gives_numerical_error(P):
    prob = qpgen.workload("small", 4)
    st = _oracle_settings(max_rejects=1, step_boost=1e6, max_outer=3)
    res_o = O.solve(prob, st)
    s = P.Solver.from_problem(prob, **_gpu_kwargs(st))
    x, lam, info = s.solve(st.eps_abs, st.eps_rel)
    assert res_o.status == O.NUMERICAL_ERROR
    assert info["status"] == O.NUMERICAL_ERROR


def test_inner_iteration_limit_continues_outer(P):
    prob = qpgen.workload("small", 5)
    st = _oracle_settings(max_inner=5, max_outer=30)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st, iters=150, trials=400)
    assert_iterate_parity(tr, t)
    assert_decision_parity(tr, t, window_of(tr))
    assert info["status"] == res_o.status == O.MAX_ITER
    assert info["outer_iters"] == 30


def test_time_limit_and_outer_limit(P):
    prob = qpgen.workload("small", 6)
    s = P.Solver.from_problem(prob, time_limit_s=0.0)
    _, _, info = s.solve(1e-4, 1e-4)
    assert info["status"] == O.TIME_LIMIT
    s2 = P.Solver.from_problem(prob, max_outer=1)
    _, _, info2 = s2.solve(1e-4, 1e-4)
    assert info2["status"] == O.MAX_ITER and info2["outer_iters"] == 1


@pytest.mark.parametrize("precision", [0, 1])
def test_kkt_pass_limit_matches_oracle(P, precision):
    """The KKT pass limit ends the solve with MAX_ITER at the same periodic
    check as the oracle (same trial count; in FP64 the same iterates)."""
    prob = qpgen.workload("small", 1)
    st = _oracle_settings(outer_scaling=2, kkt_pass_limit=300)
    res_o, tr, (x, lam, info), t, s = run_pair(P, prob, st, iters=400, trials=800,
                                               precision=precision)
    assert res_o.status == info["status"] == O.MAX_ITER
    if precision == 0:
        assert info["inner_trials"] == res_o.counters.trials
        assert_iterate_parity(tr, t)
        np.testing.assert_allclose(x, res_o.x, atol=1e-8 * max(1, np.abs(res_o.x).max()))
    assert 300 <= info["inner_trials"] < 300 + 2 * 64


def test_torch_allocator_and_stream_give_identical_results(P):
    """With torch's caching allocator and current stream plumbed in
    (settings dev_alloc/dev_free/hip_stream), a solve returns bit-identical
    results to the library's own allocations and stream, and its device
    memory comes from torch."""
    import torch
    prob = qpgen.workload("small", 2)
    kw = dict(outer_scaling=2, max_outer=20, trace_iters=200)
    s0 = P.Solver.from_problem(prob, **kw)
    x0, l0, i0 = s0.solve(1e-4, 1e-4)
    torch.cuda.reset_peak_memory_stats()
    before = torch.cuda.memory_allocated()
    s1 = P.Solver.from_problem(prob, use_torch=True, **kw)
    assert torch.cuda.memory_allocated() > before
    x1, l1, i1 = s1.solve(1e-4, 1e-4)
    assert np.array_equal(x0, x1) and np.array_equal(l0, l1)
    assert i0["inner_accepted"] == i1["inner_accepted"] and i0["status"] == i1["status"]
    assert np.array_equal(s0.trace()["w"], s1.trace()["w"])
    s1.close()
    assert torch.cuda.memory_allocated() == before


def test_warm_start_arguments(P):
    prob = qpgen.workload("small", 7)
    rng = np.random.default_rng(0)
    x0 = rng.uniform(-0.5, 1.5, prob["n"])
    l0 = rng.normal(size=prob["m"])
    st = _oracle_settings(max_outer=6, outer_scaling=2)
    tr = O.Trace(max_iters=300)
    res_o = O.solve(prob, st, x0=x0, lam0=l0, trace=tr)
    s = P.Solver.from_problem(prob, trace_iters=300, trace_trials=600, **_gpu_kwargs(st))
    x, lam, info = s.solve(st.eps_abs, st.eps_rel, x0=x0, lam0=l0)
    assert_iterate_parity(tr, s.trace())


@pytest.fixture(scope="module")
def medium_oracle():
    prob = qpgen.workload("medium", 1)
    st = _oracle_settings(max_outer=7, max_inner=256, outer_scaling=2)
    tr = O.Trace(max_iters=1000)
    res_o = O.solve(prob, st, trace=tr)
    return prob, st, tr, res_o


@pytest.mark.timeout(600)
@pytest.mark.parametrize("panels", [1, 2])
def test_medium_first_1000_iterations(P, medium_oracle, panels):
    """n = 100,000 (m = 50,000): every entry of w and y after each of the
    first 1000 accepted iterations, spanning several outer steps, stopping
    checks and restarts, at 1e-9 relative, with identical decisions; in the
    one-launch form of the first product and in the two-panel form (forced
    here: at this size x fits one XCD's L2), whose Q-row sums are formed in
    the A' epilogue."""
    prob, st, tr, res_o = medium_oracle
    s = P.Solver.from_problem(prob, trace_iters=1000, trace_trials=3000, col_panels=panels,
                              **_gpu_kwargs(st))
    s.solve(st.eps_abs, st.eps_rel)
    t = s.trace()
    assert_iterate_parity(tr, t, n_expect=1000)
    compared = assert_decision_parity(tr, t, window_of(tr))
    assert compared >= 12
    assert any(c[0] == "restart" for c in tr.checks[:compared])
    if panels == 2:
        assert "qa_panels" in {k["name"] for k in s.kernel_stats()}


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_stream_launches(P, precision):
    """With settings.graph the chunk of each outer step is captured once and
    replayed (with host reads of the control block between replays, and a
    new capture at every outer step); it runs the same kernels in the same
    order, so traces and results equal those of plain launches bit for bit."""
    prob = qpgen.workload("small", 2)
    st = _oracle_settings(max_outer=25, outer_scaling=2)
    outs = []
    for g in (0, 1):
        s = P.Solver.from_problem(prob, precision=precision, graph=g, trace_iters=500,
                                  trace_trials=2000, **_gpu_kwargs(st))
        x, lam, info = s.solve(st.eps_abs, st.eps_rel)
        outs.append((x, lam, info, s.trace()))
    (x0, l0, i0, t0), (x1, l1, i1, t1) = outs
    assert i0["outer_iters"] == i1["outer_iters"] and i0["outer_iters"] > 3
    assert i0["inner_trials"] == i1["inner_trials"]
    for key in ("w", "y", "trials", "checks"):
        assert np.array_equal(t0[key], t1[key]), key
    assert np.array_equal(x0, x1) and np.array_equal(l0, l1)


def test_anderson_steps_match_oracle(P):
    """Anderson acceleration of (lambda_E, lambda_I, z) (Section 3.2): on an
    instance whose first extrapolation comes after 1600 accepted inner
    iterations, the iterates before and after it match the oracle's at 1e-9
    (the extrapolated multipliers and centre enter every later iterate)."""
    prob = qpgen.random_indefinite_qp(300, 150, 5, 4, 1, instance=1)
    st = _oracle_settings(anderson_mem=5, outer_scaling=2, max_outer=400, eps_abs=1e-2,
                          eps_rel=1e-2)
    first = []
    tr = O.Trace(max_iters=1800)
    orig = O._anderson_outer

    def spy(*a, **k):
        out = orig(*a, **k)
        if out[2] is not None and not first:
            first.append(len(tr.w))
        return out

    O._anderson_outer = spy
    try:
        res_o = O.solve(prob, st, trace=tr)
    finally:
        O._anderson_outer = orig
    assert first and first[0] < 1700, "the oracle extrapolates inside the window"
    s = P.Solver.from_problem(prob, trace_iters=1800, trace_trials=8000, **_gpu_kwargs(st))
    x, lam, info = s.solve(st.eps_abs, st.eps_rel)
    assert_iterate_parity(tr, s.trace(), n_expect=1800)
    assert info["anderson_steps"] >= 1
    assert info["status"] == res_o.status == O.SOLVED
