"""GPU parity of the batched persistent solve (pdnqp_solve_batch: one kernel
launch, one workgroup per instance at a time) against the FP64 CPU oracle,
instance by instance, on uneven batches drawn like the batched workload
(n_i ~ U{lo..hi}, m_i = n_i // 2, k_R = 5, k_A = 4).

FP64: the first accepted iterations of every instance match the oracle's at
1e-9 relative, with identical accept/reject and check decisions inside that
window, for each workgroup size.  Full solves: same status as the oracle,
termination test met, reported KKT residuals those of the returned point.
FP32 bulk: iterates track the oracle at 1e-4 over the first iterations and
the instances solve to the tolerance.
"""

import numpy as np
import pytest

import qpgen
from oracle import pdnqp_oracle as O
from tests.test_gpu_parity import (EDGE, _gpu_kwargs, assert_decision_parity,
                                   assert_iterate_parity, assert_meets_tolerance, window_of)

pytestmark = pytest.mark.gpu

ITERS = 1000


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    P.load()
    return P


def _batch(seed, count, lo, hi):
    sizes = qpgen.batch_sizes(seed, count, lo, hi)
    return [qpgen.random_indefinite_qp(int(n), int(n) // 2, 5, 4, seed, instance=i)
            for i, n in enumerate(sizes)]


@pytest.fixture(scope="module")
def parity_case():
    probs = _batch(7, 5, 200, 1200)
    st = O.Settings(max_outer=30, outer_scaling=2)  # at least 1000 accepted iterations each
    traces = []
    for p in probs:
        tr = O.Trace(max_iters=ITERS)
        O.solve(p, st, trace=tr)
        traces.append(tr)
    return probs, st, traces


def _solve_batch(P, probs, st, config=(0, 1), **kw):
    solvers = [P.Solver.from_problem(p, **_gpu_kwargs(st), **kw) for p in probs]
    P.batch_set_config(*config)
    try:
        out = P.solve_batch(solvers, st.eps_abs, st.eps_rel)
    finally:
        P.batch_set_config(0)
    return solvers, out, P.batch_report(len(probs))


@pytest.mark.parametrize("config", [(256, 1), (512, 1), (1024, 1), (256, 4), (512, 4)])
def test_batch_fp64_iterates_match_oracle(P, parity_case, config):
    probs, st, traces = parity_case
    solvers, out, rep = _solve_batch(P, probs, st, config, trace_iters=ITERS,
                                     trace_trials=4 * ITERS)
    assert (rep["block"], rep["waves"]) == config and rep["count"] == len(probs)
    assert rep["staged"] == len(probs)  # small instances fit in LDS
    for k, (p, s, tr) in enumerate(zip(probs, solvers, traces)):
        t = s.trace()
        assert_iterate_parity(tr, t, n_expect=min(ITERS, len(tr.w)))
        assert_decision_parity(tr, t, window_of(tr))
        assert out[k][2]["gamma"] == pytest.approx(tr_gamma(p, st), rel=1e-10)


_GAMMA = {}


def tr_gamma(p, st):
    key = (p["n"], p["seed"], p.get("instance"))
    if key not in _GAMMA:
        _GAMMA[key] = O.solve(p, O.Settings(max_outer=0, outer_scaling=st.outer_scaling)).gamma
    return _GAMMA[key]


def test_batch_fp64_unstaged_matches_oracle(P, parity_case):
    """An instance too large to stage in LDS runs with global gathers; its
    first iterations still match the oracle."""
    prob = qpgen.random_indefinite_qp(30000, 15000, 5, 4, 3, instance=0)
    st = O.Settings(max_outer=2, max_inner=80, outer_scaling=2)
    tr = O.Trace(max_iters=60)
    O.solve(prob, st, trace=tr)
    solvers, out, rep = _solve_batch(P, [prob], st, (256, 1), trace_iters=60, trace_trials=200)
    assert rep["staged"] == 0
    t = solvers[0].trace()
    assert_iterate_parity(tr, t, n_expect=60)
    assert_decision_parity(tr, t, window_of(tr))


def test_batch_large_next_to_small(P):
    """One launch with a large unstaged instance (n = 70000) next to small
    staged ones: each follows the oracle."""
    probs = [qpgen.random_indefinite_qp(70000, 35000, 5, 4, 4, instance=0),
             qpgen.random_indefinite_qp(500, 250, 5, 4, 4, instance=1),
             qpgen.random_indefinite_qp(900, 450, 5, 4, 4, instance=2)]
    st = O.Settings(max_outer=2, max_inner=64, outer_scaling=2)
    solvers, out, rep = _solve_batch(P, probs, st, (512, 1), trace_iters=40, trace_trials=120)
    for p, s in zip(probs, solvers):
        tr = O.Trace(max_iters=40)
        O.solve(p, st, trace=tr)
        t = s.trace()
        assert_iterate_parity(tr, t, n_expect=40)
        assert_decision_parity(tr, t, window_of(tr))


def test_batch_fp64_full_solves(P):
    probs = _batch(11, 4, 200, 700)
    st = O.Settings(outer_scaling=2, max_outer=5000, time_limit=120.0)
    solvers, out, rep = _solve_batch(P, probs, st)
    for p, (x, lam, info) in zip(probs, out):
        res_o = O.solve(p, st)
        assert info["status"] == res_o.status == O.SOLVED
        assert info["r_p_scaled"] <= 1e-4 + 1e-4 * info["s_p_scaled"]
        assert info["r_d_scaled"] <= 1e-4 + 1e-4 * info["s_d_scaled"]
        assert_meets_tolerance(info, 1e-4, 1e-4)
        rp, rd, _, _ = O.external_kkt(p, x, lam)
        assert info["r_p"] == pytest.approx(rp, rel=1e-6, abs=1e-12)
        assert info["r_d"] == pytest.approx(rd, rel=1e-6, abs=1e-12)
        assert np.all(x >= p["xl"]) and np.all(x <= p["xu"])
        assert 0 < info["setup_s"] <= info["solve_s"]
    done = P.batch_report(len(probs))["done_ms"]
    assert np.all(done > 0)


def test_batch_edge_cases(P):
    """All edge-case problems (no rows, equalities only, two-sided rows,
    empty rows with free variables, one variable, ragged tails) in one
    launch; each follows the oracle's trajectory and ends like it."""
    names = sorted(EDGE)
    probs = [EDGE[k] for k in names]
    st = O.Settings(max_outer=12, outer_scaling=2)
    solvers, out, rep = _solve_batch(P, probs, st, trace_iters=400, trace_trials=800)
    for name, p, s, (x, lam, info) in zip(names, probs, solvers, out):
        tr = O.Trace(max_iters=400)
        res_o = O.solve(p, st, trace=tr)
        t = s.trace()
        assert_iterate_parity(tr, t)
        assert_decision_parity(tr, t, window_of(tr))
        assert info["status"] == res_o.status, name
        np.testing.assert_allclose(x, res_o.x, atol=1e-8 * max(1, np.abs(res_o.x).max()),
                                   err_msg=name)


def test_batch_limits(P):
    """Outer-iteration, inner-iteration and time limits end each instance
    (and so the launch); the inner limit continues the outer loop."""
    probs = _batch(5, 3, 300, 600)
    st = O.Settings(max_inner=5, max_outer=30)
    solvers, out, rep = _solve_batch(P, probs, st, trace_iters=150, trace_trials=400)
    for p, s, (x, lam, info) in zip(probs, solvers, out):
        tr = O.Trace(max_iters=150)
        res_o = O.solve(p, st, trace=tr)
        assert_iterate_parity(tr, s.trace())
        assert info["status"] == res_o.status == O.MAX_ITER
        assert info["outer_iters"] == 30
    st2 = O.Settings(time_limit=0.0)
    _, out2, _ = _solve_batch(P, probs, st2)
    assert all(o[2]["status"] == O.TIME_LIMIT for o in out2)
    # the KKT pass limit ends each instance at the oracle's check
    st3 = O.Settings(outer_scaling=2, kkt_pass_limit=250)
    _, out3, _ = _solve_batch(P, probs, st3)
    for p, (x, lam, info) in zip(probs, out3):
        res_o = O.solve(p, st3)
        assert info["status"] == res_o.status == O.MAX_ITER
        assert info["inner_trials"] == res_o.counters.trials


def test_batch_fp32_tracks_oracle_and_solves(P):
    probs = _batch(13, 4, 200, 900)
    st = O.Settings(outer_scaling=2, max_outer=5000, time_limit=120.0)
    solvers, out, rep = _solve_batch(P, probs, st, precision=P.FP32, trace_iters=40)
    for p, s, (x, lam, info) in zip(probs, solvers, out):
        tr = O.Trace(max_iters=40)
        O.solve(p, O.Settings(outer_scaling=2, max_outer=3), trace=tr)
        t = s.trace()
        for k in range(30):
            wn = max(1.0, np.abs(tr.w[k]).max())
            assert np.abs(t["w"][k] - tr.w[k]).max() / wn <= 1e-4, f"w at {k}"
        assert info["status"] == O.SOLVED
        assert_meets_tolerance(info, 1e-4, 1e-4)
        rp, rd, _, _ = O.external_kkt(p, x, lam)
        assert info["r_p"] == pytest.approx(rp, rel=1e-6, abs=1e-12)


def test_batch_rejects_mixed_precision(P):
    probs = _batch(2, 2, 200, 300)
    a = P.Solver.from_problem(probs[0], time_limit_s=10.0)
    b = P.Solver.from_problem(probs[1], precision=P.FP32, time_limit_s=10.0)
    with pytest.raises(P.PdnqpError, match="precision"):
        P.solve_batch([a, b])


def test_batch_autotune_caches_choice(P):
    probs = _batch(17, 8, 200, 2000)
    solvers = [P.Solver.from_problem(p, time_limit_s=60.0) for p in probs]
    cfg, ms = P.batch_autotune(solvers, probe_inner=32)
    assert cfg in P.BATCH_CONFIGS and len(ms) == 5 and min(ms) > 0
    assert ms[P.BATCH_CONFIGS.index(cfg)] == min(ms)
    out = P.solve_batch(solvers)
    rep = P.batch_report(len(probs))
    assert rep["tuned"] == 1 and (rep["block"], rep["waves"]) == cfg
    assert all(np.all(np.isfinite(x)) for x, _, _ in out)


def test_batch_anderson_matches_oracle(P):
    """Anderson acceleration inside the batched kernel: the same instance as
    the single-solve Anderson test, next to two others in one launch; the
    iterates before and after the first extrapolation match the oracle's."""
    probs = [qpgen.random_indefinite_qp(300, 150, 5, 4, 1, instance=1)] + _batch(23, 2, 200, 400)
    st = O.Settings(anderson_mem=5, outer_scaling=2, max_outer=400, eps_abs=1e-2, eps_rel=1e-2)
    solvers, out, rep = _solve_batch(P, probs, st, trace_iters=1800, trace_trials=8000)
    tr = O.Trace(max_iters=1800)
    res_o = O.solve(probs[0], st, trace=tr)
    assert res_o.anderson_steps >= 1
    assert_iterate_parity(tr, solvers[0].trace(), n_expect=1800)
    assert out[0][2]["anderson_steps"] >= 1
    assert out[0][2]["status"] == res_o.status == O.SOLVED
    assert_meets_tolerance(out[0][2], 1e-2, 1e-2)
    for p, (x, lam, info) in zip(probs[1:], out[1:]):
        assert info["status"] == O.solve(p, st).status
