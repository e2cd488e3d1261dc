"""The oracle against its stored reference values (tests/golden/), written by
tests/golden/make_golden.py from the oracle alone.  A failure here means the
oracle's arithmetic changed; such a change must name the passage of the
paper, or the reading of it, that justifies it, and regenerate the file."""

import json
import os

import numpy as np
import pytest

from tests.golden.make_golden import small_seed1

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def stored():
    with open(os.path.join(HERE, "oracle_small_seed1.json")) as f:
        return json.load(f)


def test_oracle_reproduces_stored_trajectory(stored):
    now = small_seed1()
    assert now["gamma"] == pytest.approx(stored["gamma"], rel=1e-12)
    assert now["lambda_hat"] == pytest.approx(stored["lambda_hat"], rel=1e-12)
    assert (now["status"], now["outer_iters"], now["accepted"]) == \
        (stored["status"], stored["outer_iters"], stored["accepted"])
    for key in ("w_inf", "w_sum", "y_inf"):
        np.testing.assert_allclose(now[key], stored[key], rtol=1e-10, atol=1e-12, err_msg=key)
    a_now = [t[2] for t in now["trials_lr"]]
    a_old = [t[2] for t in stored["trials_lr"]]
    assert a_now == a_old
    np.testing.assert_allclose([t[:2] for t in now["trials_lr"]],
                               [t[:2] for t in stored["trials_lr"]], rtol=1e-10, atol=1e-14)
    assert now["objective"] == pytest.approx(stored["objective"], rel=1e-9)
