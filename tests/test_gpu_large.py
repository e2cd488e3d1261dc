"""Full-size runs (n about 1M).

Parity at the benchmark's full size: the large workload (n = 1,000,000,
m = 500,000, nnz(Q) = 5M, nnz(A) = 4M, seed 1) in the launch configuration
the benchmark times (default settings), against the FP64 oracle over the
first 260 accepted inner iterations of the first outer step (inner limit
260, initial inner tolerance 1e-12 so that the stopping test does not end
it): four stopping/restart checks on the full-size check kernels (the first
ends in a restart with a primal-weight update and a step rebuild) and the
check at the inner limit.

FP64: every recorded iterate (w and y, all 2.25M entries each) matches at
1e-9 relative, with identical accept/reject and check decisions.  FP32 bulk:
the same iterates at 1e-4.  Both: the library's final KKT report equals the
oracle's formula evaluated on the returned point.

Time to tolerance at full size on the flow-family stand-in (999,990 arcs):
full solves to 1e-4 in FP64, and in FP32 bulk through its hand-over to FP64.
"""

import numpy as np
import pytest

import qpgen
from oracle import pdnqp_oracle as O
from tests.test_gpu_parity import (_gpu_kwargs, assert_decision_parity, assert_iterate_parity,
                                   assert_meets_tolerance, window_of)

pytestmark = pytest.mark.gpu

ITERS = 260


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def large_case():
    prob = qpgen.workload("large", 1)
    st = O.Settings(max_outer=1, max_inner=ITERS, delta0=1e-12)
    tr = O.Trace(max_iters=ITERS)
    res = O.solve(prob, st, trace=tr)
    return prob, st, tr, res


def _run(P, prob, st, precision):
    s = P.Solver.from_problem(prob, trace_iters=ITERS, trace_trials=4 * ITERS,
                              precision=precision, profile=32, **_gpu_kwargs(st))
    x, lam, info = s.solve(st.eps_abs, st.eps_rel)
    return s, x, lam, info


def _check_report(prob, x, lam, info):
    rp, rd, sp_, sd = O.external_kkt(prob, x, lam)
    assert info["r_p"] == pytest.approx(rp, rel=1e-6, abs=1e-12)
    assert info["r_d"] == pytest.approx(rd, rel=1e-6, abs=1e-12)
    assert np.all(x >= prob["xl"]) and np.all(x <= prob["xu"])


@pytest.mark.timeout(900)
def test_large_fp64_first_iterations(P, large_case):
    prob, st, tr, res = large_case
    assert len(tr.w) == ITERS
    s, x, lam, info = _run(P, prob, st, P.FP64)
    t = s.trace()
    assert_iterate_parity(tr, t, n_expect=ITERS)
    compared = assert_decision_parity(tr, t, window_of(tr))
    assert compared == 5 and tr.checks[0][0] == "restart"
    assert info["status"] == res.status
    np.testing.assert_allclose(x, res.x, atol=1e-9 * max(1.0, np.abs(res.x).max()))
    _check_report(prob, x, lam, info)


@pytest.mark.timeout(600)
def test_large_fp32_first_iterations(P, large_case):
    prob, st, tr, res = large_case
    s, x, lam, info = _run(P, prob, st, P.FP32)
    t = s.trace()
    assert t["w"].shape[0] == ITERS
    for k in range(ITERS):
        W, Y = np.asarray(tr.w[k]), np.asarray(tr.y[k])
        dw = np.abs(t["w"][k] - W).max() / max(1.0, np.abs(W).max())
        dy = np.abs(t["y"][k] - Y).max() / max(1.0, np.abs(Y).max())
        assert dw <= 1e-4 and dy <= 1e-4, (k, dw, dy)
    assert info["status"] == res.status
    _check_report(prob, x, lam, info)


@pytest.fixture(scope="module")
def flow_case():
    return qpgen.flow_qp(101)


def test_flow_family_million_solves(P, flow_case):
    """The flow-family stand-in at n = 999,990 arcs (m = 355,552 node rows)
    from its feasible reference flow: FP64 reaches the 1e-4 test, and the
    library's KKT report is the oracle's formula on the returned point."""
    prob = flow_case
    s = P.Solver.from_problem(prob, time_limit_s=120.0)
    x, lam, info = s.solve(1e-4, 1e-4, x0=prob["x0"])
    assert info["status"] == O.SOLVED
    assert info["r_p_scaled"] <= 1e-4 + 1e-4 * info["s_p_scaled"]
    assert info["r_d_scaled"] <= 1e-4 + 1e-4 * info["s_d_scaled"]
    assert_meets_tolerance(info, 1e-4, 1e-4)
    _check_report(prob, x, lam, info)
    print(f"flow n={prob['n']}: {info['solve_s']:.2f} s, {info['outer_iters']} outer, "
          f"{info['inner_accepted']} inner")


def test_flow_family_fp32_promotes_on_stall(P, flow_case):
    """FP32 bulk stalls above the tolerance on this instance (its rounding
    keeps the dual residual near 3e-3); after 50 outer steps without a 10%
    gain it hands over to the FP64 inner iteration and the solve succeeds."""
    prob = flow_case
    s = P.Solver.from_problem(prob, precision=P.FP32, time_limit_s=120.0)
    x, lam, info = s.solve(1e-4, 1e-4, x0=prob["x0"])
    assert info["status"] == O.SOLVED
    assert_meets_tolerance(info, 1e-4, 1e-4)
    assert info["promoted_outer"] > 0
    _check_report(prob, x, lam, info)
    print(f"flow n={prob['n']} FP32: promoted at outer step {info['promoted_outer']}, "
          f"{info['solve_s']:.2f} s, {info['outer_iters']} outer")
