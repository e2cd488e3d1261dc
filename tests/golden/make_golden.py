"""Writes the oracle's reference values stored beside this script.

Run from the repository root:  python tests/golden/make_golden.py

Only the oracle (oracle/pdnqp_oracle.py) and the seeded generator produce the
values; nothing here comes from the GPU path.  A change of these files must
come with a change of the oracle's arithmetic whose commit names the passage
of the paper (or the reading of it) that justifies it.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import qpgen  # noqa: E402
from oracle import pdnqp_oracle as O  # noqa: E402

ITERS = 40


def small_seed1():
    """Small workload, seed 1, Q-aware outer scaling, 6 outer steps: the
    first ITERS accepted inner iterates (their infinity norms and sums),
    every trial's acceptance sums, the proximal step and the result."""
    prob = qpgen.workload("small", 1)
    st = O.Settings(max_outer=6, outer_scaling=2)
    tr = O.Trace(max_iters=ITERS)
    res = O.solve(prob, st, trace=tr)
    return {
        "instance": "qpgen.workload('small', 1); Settings(max_outer=6, outer_scaling=2)",
        "gamma": res.gamma,
        "lambda_hat": res.lambda_hat,
        "status": res.status,
        "outer_iters": res.outer_iters,
        "accepted": res.counters.accepted,
        "w_inf": [float(np.abs(w).max()) for w in tr.w],
        "w_sum": [float(np.sum(w)) for w in tr.w],
        "y_inf": [float(np.abs(y).max()) for y in tr.y],
        "trials_lr": [[float(l), float(r), bool(a)] for (l, r, a) in tr.trials[:ITERS]],
        "x_sum": float(np.sum(res.x)),
        "objective": res.objective,
    }


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small_seed1.json")
    with open(out, "w") as f:
        json.dump(small_seed1(), f, indent=1)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
