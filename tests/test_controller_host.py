"""Host-side pieces of the learned controller (no GPU): hindsight labels,
folding the feature standardisation into the first layer, SGM10."""

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2609_19557_amd import controller as C


def test_hindsight_labels_read_the_next_step():
    # records: r_p, r_d, s_p, s_d, omega_end, inner, restarts, delta_used
    rec = np.array([[1.0, 0.5, 2.0, 4.0, 0.3, 100, 2, 1.0],
                    [0.2, 0.4, 2.0, 4.0, 0.5, 640, 5, 0.3],
                    [1e-6, 1e-6, 2.0, 4.0, 0.7, 64, 0, 0.09]])
    feat = np.arange(48, dtype=float).reshape(3, 16)
    X, Y = C.hindsight_labels(feat, rec, eps=1e-4, check_every=64)
    assert X.shape == (2, 16) and Y.shape == (2, 3)
    np.testing.assert_array_equal(X, feat[:2])
    # step 1: max(0.2/2, 0.4/4) = 0.1 -> delta* = 0.01; budget 2*640+64; omega 0.5
    np.testing.assert_allclose(Y[0], [np.log(0.01), np.log(1344.0), np.log(0.5)])
    # step 2: tiny residual -> delta* floored at eps
    np.testing.assert_allclose(Y[1], [np.log(1e-4), np.log(192.0), np.log(0.7)])


def test_hindsight_labels_need_two_steps():
    X, Y = C.hindsight_labels(np.zeros((1, 16)), np.ones((1, 8)))
    assert X.shape == (0, 16) and Y.shape == (0, 3)


def test_fold_normalisation_is_exact():
    """The network on raw features with the folded parameters equals the
    network on standardised features."""
    rng = np.random.default_rng(6)
    th = rng.normal(scale=0.25, size=M.N_PARAMS)
    X = rng.normal(size=(50, 16))
    mu = X.mean(axis=0)
    sd = X.std(axis=0) + 0.5
    y_std, _ = M.forward(th, (X - mu) / sd)
    y_raw, _ = M.forward(C.fold_normalisation(th, mu, sd).astype(np.float64), X)
    np.testing.assert_allclose(y_raw, y_std, rtol=1e-5, atol=1e-5)


def test_sgm10_definition():
    """eq. (sgm10): exp(mean log(t + 10)) - 10."""
    assert C.sgm10([0.0]) == pytest.approx(0.0)
    assert C.sgm10([10.0, 30.0]) == pytest.approx(np.sqrt(20.0 * 40.0) - 10.0)


def test_committed_weights_shape():
    th = C.load_weights()
    assert th.dtype == np.float32 and th.shape == (M.N_PARAMS,) and np.all(np.isfinite(th))
