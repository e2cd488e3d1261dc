"""Learned outer-step controller: data collection, hindsight labels and
training, on top of the library's outer-step log and its GPU network
kernels (``mlp_train``).

At the end of each outer step the controller sees 16 features (the library
records them with ``settings.outer_log``) and sets, for the next inner
solve, the inner tolerance delta, an iteration budget K (reaching it ends
the inner solve) and the starting primal weight omega.  It replaces the
adaptive inner-tolerance rule (inner-tolerance-factor) until three outer
steps pass without progress of the outer KKT measure; the library then
falls back to that rule for the rest of the solve.

Hindsight labels, from trajectories of the plain method: for the features
of step k, the targets describe step k + 1 as it turned out --
    log delta* = log max(eps, c_delta * max(r_p / s_p, r_d / s_d)_{k+1})
    log K*     = log(2 * (accepted inner iterations)_{k+1} + check_every)
    log omega* = log(primal weight at the end of step k+1's inner solve)
i.e. an inner tolerance a fraction of the outer residual the next step
reached, a budget with room over the iterations it needed, and the primal
weight it settled at.
"""

from __future__ import annotations

import os

import numpy as np

from . import pdnqp as _p

FEATURE_NAMES = ["log r_p", "log r_d", "log s_p", "log s_d", "log |x-z|/gamma", "log delta_a",
                 "log eps_a,k", "log omega", "log min sigma", "log mean sigma",
                 "log max sigma", "log r_p/r_p,prev", "log r_d/r_d,prev", "log 1+inner",
                 "log 1+restarts", "log 1+k"]
C_DELTA = 0.1
WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "controller_weights.npy")


def hindsight_labels(feat, rec, eps=1e-4, check_every=64):
    """(X, Y) pairs from one recorded trajectory: features of steps
    0..T-2 and the targets read off steps 1..T-1."""
    feat = np.asarray(feat, dtype=np.float64)
    rec = np.asarray(rec, dtype=np.float64)
    if feat.shape[0] < 2:
        return np.zeros((0, 16)), np.zeros((0, 3))
    nxt = rec[1:]
    rel = np.maximum(nxt[:, 0] / nxt[:, 2], nxt[:, 1] / nxt[:, 3])
    y_delta = np.log(np.maximum(eps, C_DELTA * rel))
    y_budget = np.log(2.0 * nxt[:, 5] + check_every)
    y_omega = np.log(np.maximum(nxt[:, 4], 1e-12))
    return feat[:-1], np.stack([y_delta, y_budget, y_omega], axis=1)


def collect(problems, eps=1e-4, max_log=4000, **settings):
    """Plain solves (adaptive rule) of ``problems`` with the outer log on;
    returns stacked (X, Y) and per-problem solve reports."""
    Xs, Ys, infos = [], [], []
    for prob in problems:
        s = _p.Solver.from_problem(prob, outer_log=max_log, **settings)
        _, _, info = s.solve(eps, eps)
        f, r = s.outer_log()
        X, Y = hindsight_labels(f, r, eps=eps, check_every=s.settings.check_every)
        Xs.append(X)
        Ys.append(Y)
        infos.append(info)
        s.close()
    return np.concatenate(Xs), np.concatenate(Ys), infos


def init_theta(seed):
    """He-style initial parameters."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in [(16, 64), (64,), (64, 64), (64,), (64, 3), (3,)]:
        if len(shape) == 2:
            parts.append(rng.normal(scale=np.sqrt(2.0 / shape[0]), size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def fold_normalisation(theta, mu, sd):
    """Parameters of the network applied to raw features from those of the
    network applied to (x - mu) / sd: W1' = W1 / sd, b1' = b1 - (mu / sd) W1."""
    th = np.array(theta, dtype=np.float64, copy=True)
    W1 = th[:16 * 64].reshape(16, 64)
    b1 = th[16 * 64:16 * 64 + 64]
    th[16 * 64:16 * 64 + 64] = b1 - (mu / sd) @ W1
    th[:16 * 64] = (W1 / sd[:, None]).ravel()
    return th.astype(np.float32)


def train(X, Y, seed=0, epochs=300, batch=128, lr=2e-3):
    """Trains on the GPU (the library's Adam loop) on standardised features
    and returns parameters for raw features and the loss curve."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    th, curve = _p.mlp_train(init_theta(seed), (X - mu) / sd, Y, epochs=epochs,
                             batch=min(batch, X.shape[0]), lr=lr, seed=seed)
    return fold_normalisation(th, mu, sd), curve


def load_weights(path=WEIGHTS_FILE):
    """Committed parameters (``python -m paper_2609_19557_amd.controller``)."""
    return np.load(path, allow_pickle=False).astype(np.float32)


def sgm10(times):
    """Shifted geometric mean with a 10-second shift (the paper's SGM10)."""
    t = np.asarray(times, dtype=np.float64)
    return float(np.exp(np.mean(np.log(t + 10.0))) - 10.0)


def _main():
    import argparse
    import json
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import qpgen
    ap = argparse.ArgumentParser(description="train the controller on plain trajectories")
    ap.add_argument("--train-seeds", type=int, default=48)
    ap.add_argument("--eval-seeds", type=int, default=12)
    ap.add_argument("--out", default=WEIGHTS_FILE)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    _p.load()
    kw = dict(outer_scaling=_p.SCALE_RUIZ_QA, time_limit_s=60.0)
    train_probs = [qpgen.random_indefinite_qp(n, n // 2, 5, 4, 1000 + i)
                   for i, n in enumerate(np.geomspace(300, 3000, args.train_seeds).astype(int))]
    X, Y, _ = collect(train_probs, **kw)
    theta, curve = train(X, Y)
    np.save(args.out, theta)
    rows = []
    for i, n in enumerate(np.geomspace(300, 3000, args.eval_seeds).astype(int)):
        prob = qpgen.random_indefinite_qp(int(n), int(n) // 2, 5, 4, 2000 + i)
        res = {}
        for ctl in (0, 1):
            s = _p.Solver.from_problem(prob, controller=ctl, **kw)
            if ctl:
                s.set_controller(theta)
            _, _, info = s.solve(1e-4, 1e-4)
            res[ctl] = info
            s.close()
        rows.append({"n": int(n), "plain": [res[0]["status"], res[0]["inner_accepted"],
                                            round(res[0]["solve_s"], 3)],
                     "learned": [res[1]["status"], res[1]["inner_accepted"],
                                 round(res[1]["solve_s"], 3), res[1]["controller_fallback"]]})
    rep = {"samples": int(X.shape[0]), "final_loss": float(curve[-1]), "eval": rows}
    print(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    _main()
