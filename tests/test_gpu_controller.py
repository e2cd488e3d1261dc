"""Learned outer-step controller on the GPU: the network's forward pass and
gradient against the FP64 CPU reference (oracle/mlp_oracle.py), training,
the outer-step log against the oracle's outer trace, and the controller's
fallback to the adaptive rule."""

import numpy as np
import pytest

import qpgen
from oracle import mlp_oracle as M
from oracle import pdnqp_oracle as O
from tests.test_gpu_parity import _gpu_kwargs, assert_meets_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    P.load()
    return P


def _data(seed, count):
    rng = np.random.default_rng(seed)
    th = rng.normal(scale=0.25, size=M.N_PARAMS)
    X = rng.normal(size=(count, 16))
    Y = rng.normal(size=(count, 3))
    return th, X, Y


def test_mlp_forward_matches_cpu(P):
    th, X, _ = _data(1, 300)
    y_gpu = P.mlp_forward(th, X)
    y_cpu, _ = M.forward(th.astype(np.float32).astype(np.float64),
                         X.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(y_gpu, y_cpu, rtol=2e-5, atol=2e-5)


@pytest.mark.parametrize("count", [1, 63, 64, 65, 1000])
def test_mlp_gradient_matches_cpu(P, count):
    """FP32 gradient over ragged sample counts (partial workgroups) against
    the FP64 chain rule on the same FP32-rounded inputs."""
    th, X, Y = _data(2, count)
    th32 = th.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    Y32 = Y.astype(np.float32).astype(np.float64)
    g_gpu, l_gpu = P.mlp_gradient(th, X, Y)
    g_cpu = M.gradient(th32, X32, Y32)
    assert l_gpu == pytest.approx(M.loss(th32, X32, Y32), rel=1e-5)
    err = np.abs(g_gpu - g_cpu).max() / max(1e-12, np.abs(g_cpu).max())
    assert err <= 1e-4, err


def test_mlp_training_fits_teacher(P):
    """Adam on the GPU fits targets made by a random teacher network."""
    rng = np.random.default_rng(3)
    teacher = rng.normal(scale=0.3, size=M.N_PARAMS)
    X = rng.normal(size=(2000, 16))
    Y, _ = M.forward(teacher, X)
    from paper_2609_19557_amd import controller as C
    th0 = C.init_theta(4)
    l0 = M.loss(th0.astype(np.float64), X, Y)
    th, curve = P.mlp_train(th0, X, Y, epochs=60, batch=128, lr=2e-3, seed=5)
    assert curve[-1] < 0.1 * l0
    assert M.loss(th.astype(np.float64), X, Y) == pytest.approx(curve[-1], rel=1e-3)


def test_outer_log_matches_oracle(P):
    """The logged outer residuals of the first outer steps are the oracle's
    (inside the iterate-parity window), and the features are the logs of
    the logged raw values."""
    prob = qpgen.workload("small", 1)
    st = O.Settings(max_outer=8, outer_scaling=2)
    tr = O.Trace(max_iters=0)
    O.solve(prob, st, trace=tr)
    s = P.Solver.from_problem(prob, outer_log=50, **_gpu_kwargs(st))
    _, _, info = s.solve(st.eps_abs, st.eps_rel)
    f, r = s.outer_log()
    assert info["outer_logged"] == f.shape[0] == len(tr.outer) == 8
    for k in range(4):
        _, rp, rd, sp_, sd = tr.outer[k]
        np.testing.assert_allclose(r[k, :4], [rp, rd, sp_, sd], rtol=1e-7)
    np.testing.assert_allclose(f[:, 0], np.log10(np.maximum(r[:, 0], 1e-30)), rtol=1e-12)
    np.testing.assert_allclose(f[:, 1], np.log10(np.maximum(r[:, 1], 1e-30)), rtol=1e-12)
    np.testing.assert_allclose(f[:, 13], np.log10(1.0 + r[:, 5]), rtol=1e-12)
    np.testing.assert_allclose(f[1:, 11], np.diff(np.log10(r[:, 0])), atol=1e-12)


def test_controller_falls_back_to_adaptive_rule(P):
    """A controller that asks for a useless inner tolerance (delta = 1) and
    the smallest budget stops the outer progress; after three steps without
    progress the adaptive rule takes over and the solve still succeeds."""
    from paper_2609_19557_amd import controller as C
    th = np.zeros(M.N_PARAMS, dtype=np.float32)
    th[-3:] = [0.0, 0.0, 0.0]   # outputs log delta = 0, log K = 0 (clamped up), log omega = 0
    prob = qpgen.workload("small", 2)
    s = P.Solver.from_problem(prob, controller=1, outer_scaling=2, time_limit_s=60.0)
    s.set_controller(th)
    _, _, info = s.solve(1e-4, 1e-4)
    assert info["controller_fallback"] == 1
    assert info["status"] == O.SOLVED
    assert_meets_tolerance(info, 1e-4, 1e-4)
    assert C.sgm10([0.0, 0.0]) == pytest.approx(0.0)


def test_controller_gain_on_held_out_seeds(P):
    """The committed controller (trained by ``python -m
    paper_2609_19557_amd.controller`` on 48 trajectories of seeds
    1000-1047) against the adaptive rule on the 12 held-out seeds 2000-2011
    of that command's evaluation: both solve every instance, and the
    controller needs fewer accepted inner iterations in geometric mean
    (the counts are deterministic)."""
    from paper_2609_19557_amd import controller as C
    theta = C.load_weights()
    kw = dict(outer_scaling=P.SCALE_RUIZ_QA, time_limit_s=60.0)
    plain, learned = [], []
    for i, n in enumerate(np.geomspace(300, 3000, 12).astype(int)):
        prob = qpgen.random_indefinite_qp(int(n), int(n) // 2, 5, 4, 2000 + i)
        a = P.Solver.from_problem(prob, **kw)
        _, _, ia = a.solve(1e-4, 1e-4)
        b = P.Solver.from_problem(prob, controller=1, **kw)
        b.set_controller(theta)
        _, _, ib = b.solve(1e-4, 1e-4)
        assert ia["status"] == ib["status"] == O.SOLVED
        assert_meets_tolerance(ia, 1e-4, 1e-4)
        assert_meets_tolerance(ib, 1e-4, 1e-4)
        plain.append(ia["inner_accepted"])
        learned.append(ib["inner_accepted"])
    gm = lambda v: float(np.exp(np.mean(np.log(v))))
    print(f"geometric-mean inner iterations: adaptive rule {gm(plain):.0f}, "
          f"learned controller {gm(learned):.0f}")
    assert gm(learned) < gm(plain)
