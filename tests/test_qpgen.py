"""The seeded input generators: the structure each family promises (CPU)."""

import numpy as np
import pytest

import qpgen
from oracle import pdnqp_oracle as O


def test_random_indefinite_large_sizes():
    """The large workload's stated totals: about 5M nonzeros in Q and 4M in A
    at n = 1M (2 entries per row of R, 8 per row of A), rows distinct."""
    p = qpgen.workload("large", 1)
    assert p["Q"].shape == (1_000_000, 1_000_000) and p["A"].shape == (500_000, 1_000_000)
    assert abs(p["Q"].nnz - 5_000_000) < 5_000 and p["A"].nnz == 4_000_000
    assert (abs(p["Q"] - p["Q"].T)).max() == 0.0
    assert np.all(np.diff(p["A"].indptr) == 8)


@pytest.mark.parametrize("seed", [101, 102, 103])
def test_flow_structure(seed):
    p = qpgen.flow_qp(seed, n_target=30_000)
    L, w = p["layers"], p["width"]
    assert L in (4, 6, 8, 12, 16)
    assert p["n"] == 3 * w * (L - 1) and p["m"] == L * w
    B = p["A"].tocsc()
    # every arc leaves one node and enters one node of the next layer
    assert np.all(np.diff(B.indptr) == 2)
    assert np.all(B.data[0::2] + B.data[1::2] == 0.0)
    heads = B.indices[1::2] // w
    tails = B.indices[0::2] // w
    assert np.all(np.abs(heads - tails) == 1)
    # the frozen start is feasible and strictly inside the capacities
    f0 = p["x0"]
    assert np.array_equal(p["rl"], p["ru"])
    assert np.abs(p["A"] @ f0 - p["rl"]).max() == 0.0
    assert np.all(f0 > 0.0) and np.all(f0 < p["xu"])
    # concave costs: Q = diag(-2 alpha c / u) < 0, c > 0
    d = p["Q"].diagonal()
    assert p["Q"].nnz == p["n"] and np.all(d < 0.0) and np.all(p["c"] > 0.0)
    np.testing.assert_allclose(d, -2.0 * p["alpha"] * p["c"] / p["xu"], rtol=1e-15)
    # the marginal cost c (1 - 2 alpha f / u) stays positive over [0, u]
    assert np.all(p["c"] * (1.0 - 2.0 * p["alpha"]) > 0.0)


def test_flow_small_instance_solves_on_the_oracle():
    """The oracle solves a small flow instance from its reference flow to a
    point whose unscaled dual residual is small in absolute terms too: with
    the penalty cap reading (1e4) the multipliers stay bounded.  (With a 1e9
    cap the penalties reached 8e8, the multipliers 5e4, and the relative test
    accepted an absolute dual residual of 2.2.)"""
    p = qpgen.flow_qp(101, n_target=3000)
    res = O.solve(p, O.Settings(time_limit=120.0), x0=p["x0"])
    assert res.status == O.SOLVED
    rp, rd, sp_, sd = O.external_kkt(p, res.x, res.lam)
    assert rd <= 1e-3 and sd <= 10.0
    assert np.abs(res.lam).max() <= 100.0
