"""Pins of the oracle's outer-loop rules, primal weight, diagonal steps and
row normalisation against what the paper states and against hand-computed
examples (none of them re-evaluates the oracle's own formula):

* primal weight (Section 3.3, eq. (primal-weight-update)): Delta_y/Delta_w
  is its fixed point, log(omega) moves exactly a quarter of the way towards
  it (hand values), a zero movement keeps omega, and along a real inner
  solve every restart moves omega towards the movement ratio;
* inner-tolerance factor (Section 3.2, eq. (inner-tolerance-factor)): 0.95
  when the proximal term vanishes, 0.3 when it dominates r_d, the midpoint
  when it is half of r_d;
* penalty trigger (Section 3.2, eq. (penalty-trigger-eq)): a hand example
  in which each row takes a different branch, the cap, the gate reading,
  and along real runs: sigma never decreases and only rows whose residual
  did not fall to 0.25 of the previous one (equality rows and active
  inequality rows) grow;
* centre update (Section 3.2, eq. (center-update)/(center-tolerance-update)):
  z moves exactly when r_p <= eps_a,k + eps_r,k s_p, and the tolerances
  then shrink by exactly rho_z, on hand cases and along real runs with the
  paper's literal rules;
* diagonal scales and steps (Section 3.3, eq. (diagonal-scales)/
  (diagonal-steps)) on a hand-built inner QP with hand-computed m_w, m_y,
  and the direction in which omega moves the two steps;
* row normalisation: tiny QPs with upper-bound and two-sided rows end at an
  enumerated KKT point with multipliers in the caller's sign convention;
* mutation checks: each plausible mistake below makes a pin fail.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from oracle import pdnqp_oracle as O
from tests.kkt_enum import kkt_points_general


# ---------------------------------------------------------------------------
# primal weight, eq. (primal-weight-update)
# ---------------------------------------------------------------------------

def _weight_pins_hold():
    f = O.primal_weight_update
    ok = True
    # the balancing ratio is a fixed point
    ok &= f(2.5, 1.0, 2.5) == pytest.approx(2.5, rel=1e-14)
    ok &= f(0.04, 3.0, 0.12) == pytest.approx(0.04, rel=1e-14)
    # a quarter of the way in log space: omega = 1, ratio 16 -> 16^(1/4) = 2;
    # omega = 8, ratio 1/2 -> exp(0.25 ln(1/2) + 0.75 ln 8) = 2^(-1/4 + 9/4) = 4
    ok &= f(1.0, 1.0, 16.0) == pytest.approx(2.0, rel=1e-14)
    ok &= f(8.0, 2.0, 1.0) == pytest.approx(4.0, rel=1e-14)
    # a zero movement keeps omega (the update needs both movements nonzero)
    ok &= f(3.0, 0.0, 1.0) == 3.0 and f(3.0, 1.0, 0.0) == 3.0
    return bool(ok)


def test_primal_weight_update_hand_values():
    assert _weight_pins_hold()


def test_primal_weight_moves_towards_movement_ratio_in_inner_solve():
    """Every restart of a real inner solve moves log(omega) towards
    log(Delta_y / Delta_w), closing exactly three quarters of the gap's
    complement (the remaining gap is 0.75 of the old one)."""
    prob = qpgen.workload("small", 2)
    tr = O.Trace()
    O.solve(prob, O.Settings(max_outer=10), trace=tr)
    moved = 0
    for w0, w1, d_w, d_y in tr.weights:
        if d_w > 0 and d_y > 0:
            target = math.log(d_y / d_w)
            gap0 = target - math.log(w0)
            gap1 = target - math.log(w1)
            assert gap1 == pytest.approx(0.75 * gap0, rel=1e-9, abs=1e-12)
            moved += 1
        else:
            assert w1 == w0
    assert moved >= 3


# ---------------------------------------------------------------------------
# inner-tolerance factor, eq. (inner-tolerance-factor)
# ---------------------------------------------------------------------------

def _tolerance_factor_pins_hold():
    st = O.Settings()
    f = O.inner_tolerance_factor
    z = np.array([0.2, 0.5, 0.9])
    ok = True
    # no proximal term: the slow factor rho_max = 0.95
    ok &= f(z.copy(), z, 0.1, 0.3, st) == pytest.approx(0.95, rel=1e-15)
    # proximal term gamma^-1 ||x - z|| = 0.4 / 0.1 = 4 >= r_d = 0.3: rho_min = 0.3
    x = z + np.array([0.0, -0.4, 0.1])
    ok &= f(x, z, 0.1, 0.3, st) == pytest.approx(0.3, rel=1e-15)
    # proximal term 0.015 / 0.1 = 0.15 = r_d / 2: 0.95 - 0.65 / 2 = 0.625
    x = z + np.array([0.015, 0.0, -0.01])
    ok &= f(x, z, 0.1, 0.3, st) == pytest.approx(0.625, rel=1e-12)
    return bool(ok)


def test_inner_tolerance_factor_hand_values():
    assert _tolerance_factor_pins_hold()


# ---------------------------------------------------------------------------
# row penalties, eq. (penalty-trigger-eq)
# ---------------------------------------------------------------------------

def _penalty_pins_hold():
    st = O.Settings(penalty_gate=False)
    sigma = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    r_prev = np.ones(5)
    r_new = np.array([0.5, 0.1, 0.3, 1.0, -2.0])
    # rows 0, 1 equalities; 2 and 4 active inequalities; 3 an inactive one
    active = np.array([True, True, True, False, True])
    new, trig = O.penalty_update(sigma, r_new, r_prev, active, 0.0, st)
    ok = True
    # ||r||_inf = 2, growth 10: row 0 x max(1, 2.5); row 1 fell below 0.25 of
    # its previous residual; row 2 x 1.5; row 3 inactive; row 4 x 10
    ok &= np.array_equal(trig, [True, False, True, False, True])
    ok &= np.allclose(new, [2.5, 2.0, 4.5, 4.0, 50.0], rtol=1e-15)
    # the cap
    big, _ = O.penalty_update(np.full(5, 9000.0), r_new, r_prev, active, 0.0, st)
    ok &= big[4] == st.sigma_max and big[1] == 9000.0
    # a residual exactly at 0.25 of the previous one does not trigger (strict >)
    eq, trig_eq = O.penalty_update(np.ones(1), np.array([0.25]), np.ones(1),
                                   np.array([True]), 0.0, st)
    ok &= not trig_eq[0] and eq[0] == 1.0
    # [reading] gate: rows already within the outer tolerance stay
    gated, _ = O.penalty_update(sigma, r_new, r_prev, active, 0.4,
                                O.Settings(penalty_gate=True))
    ok &= np.allclose(gated, [2.5, 2.0, 3.0, 4.0, 50.0], rtol=1e-15)
    return bool(ok)


def test_penalty_update_hand_example():
    assert _penalty_pins_hold()


def _run_rules(prob, st, steps):
    tr = O.Trace(max_rules=steps)
    st.max_outer = steps
    O.solve(prob, st, trace=tr)
    return tr.rules


def _rules_invariants_hold(rules, st):
    """Invariants of eq. (penalty-trigger-eq) and (center-update)/
    (center-tolerance-update) along a run."""
    centre_moves = 0
    grown = 0
    for rec in rules:
        sb, sa = rec["sigma_before"], rec["sigma_after"]
        if np.any(sa < sb):
            return False                      # penalties never decrease
        up = sa > sb
        if rec["r_prev"] is None:
            if np.any(up):
                return False                  # no previous residual: no update
        else:
            fell = np.abs(rec["r_row"]) <= st.theta_sigma * np.abs(rec["r_prev"])
            if np.any(up & (fell | ~rec["active"])):
                return False
            grown += int(up.sum())
        thr = rec["eps_before"][0] + rec["eps_before"][1] * rec["sp"]
        if rec["moved"] != (rec["rp"] <= thr):
            return False
        if rec["moved"]:
            centre_moves += 1
            if not np.array_equal(rec["z_new"], rec["x"]):
                return False
            want = [st.rho_z * e for e in rec["eps_before"]]
            if st.center_floor:
                want = [max(want[0], st.eps_abs), max(want[1], st.eps_rel)]
            if not np.allclose(rec["eps_after"], want, rtol=1e-15, atol=0):
                return False
        else:
            if not np.array_equal(rec["z_new"], rec["z_old"]):
                return False
            if rec["eps_after"] != rec["eps_before"]:
                return False
        # the slow factor exactly when the proximal term vanishes
        if np.array_equal(rec["x"], rec["z_old"]) != (rec["rho"] == st.rho_in_max):
            return False
        if not (st.rho_in_min <= rec["rho"] <= st.rho_in_max):
            return False
    return centre_moves > 0 and grown > 0


@pytest.mark.parametrize("literal", [False, True])
def test_outer_rules_invariants_along_a_run(literal):
    st = O.Settings(penalty_gate=not literal, center_floor=not literal)
    rules = _run_rules(qpgen.workload("small", 1), st, 40)
    assert len(rules) >= 30
    assert _rules_invariants_hold(rules, st)


def test_centre_tolerances_shrink_geometrically_under_literal_rule():
    """Without the floor reading, after j centre moves the centre
    tolerances are exactly 0.95^j."""
    st = O.Settings(penalty_gate=False, center_floor=False)
    rules = _run_rules(qpgen.workload("small", 1), st, 40)
    moves = 0
    for rec in rules:
        moves += rec["moved"]
        assert rec["eps_after"][0] == pytest.approx(0.95 ** moves, rel=1e-12)
        assert rec["eps_after"][1] == pytest.approx(0.95 ** moves, rel=1e-12)
    assert moves >= 5


# ---------------------------------------------------------------------------
# centre update, eq. (center-update)/(center-tolerance-update)
# ---------------------------------------------------------------------------

def _centre_pins_hold():
    st = O.Settings(center_floor=False)
    x = np.array([0.3, 0.7])
    z = np.array([0.1, 0.2])
    ok = True
    # r_p = 0.05 <= 0.01 + 0.02 * 2.5 = 0.06: the centre moves, tolerances x 0.95
    z1, ea, er, moved = O.center_update(x, z, 0.05, 2.5, 0.01, 0.02, st)
    ok &= moved and np.array_equal(z1, x)
    ok &= ea == pytest.approx(0.0095, rel=1e-15) and er == pytest.approx(0.019, rel=1e-15)
    # r_p = 0.07 > 0.06: nothing changes
    z2, ea, er, moved = O.center_update(x, z, 0.07, 2.5, 0.01, 0.02, st)
    ok &= (not moved) and np.array_equal(z2, z) and ea == 0.01 and er == 0.02
    # [reading] floored at the outer tolerances
    stf = O.Settings(center_floor=True, eps_abs=1e-4, eps_rel=1e-4)
    _, ea, er, moved = O.center_update(x, z, 0.0, 1.0, 1.02e-4, 5e-4, stf)
    ok &= moved and ea == 1e-4 and er == pytest.approx(4.75e-4, rel=1e-15)
    return bool(ok)


def test_centre_update_hand_cases():
    assert _centre_pins_hold()


# ---------------------------------------------------------------------------
# diagonal scales and steps, eq. (diagonal-scales)/(diagonal-steps)
# ---------------------------------------------------------------------------

def _hand_inner():
    """Inner QP with n = 2, one equality and one inequality row; columns
    (x1, x2, s1, rE1, rI1), row penalties sigma = (100, 4)."""
    B = sp.csr_matrix(np.array([[1.0, 2.0, 0.0, -1.0, 0.0],
                                [3.0, 0.0, -1.0, 0.0, -1.0]]))
    H = sp.csr_matrix(np.array([[2.0, -1.0, 0.0, 0.0, 0.0],
                                [-1.0, 3.0, 0.0, 0.0, 0.0],
                                [0.0, 0.0, 0.0, 0.0, 0.0],
                                [0.0, 0.0, 0.0, 100.0, 0.0],
                                [0.0, 0.0, 0.0, 0.0, 4.0]]))
    return H, B, np.array([100.0, 4.0])


def _diagonal_pins_hold():
    H, B, sigma = _hand_inner()
    m_w, m_y = O.diagonal_scales(H, B, sigma, 3)
    # by hand: x1: |2|+|-1| + max(1+3, sqrt(100*1 + 4*9)); x2: 1+3 + max(2, sqrt(100*4));
    # s1: 0 + max(1, sqrt(4*1)); rE1: 100 + 1; rI1: 4 + 1
    want_w = np.array([3.0 + math.sqrt(136.0), 24.0, 2.0, 101.0, 5.0])
    want_y = np.array([1.0 / want_w[0] + 4.0 / 24.0 + 1.0 / 101.0,
                       9.0 / want_w[0] + 1.0 / 2.0 + 1.0 / 5.0])
    ok = np.allclose(m_w, want_w, rtol=1e-14) and np.allclose(m_y, want_y, rtol=1e-14)
    st = O.Settings()
    tau1, eta1 = O.diagonal_steps(m_w, m_y, 1.0, st)
    tau2, eta2 = O.diagonal_steps(m_w, m_y, 2.0, st)
    # omega = 1: tau = 0.99 / m_w, eta = 0.99 / m_y; a larger primal weight
    # shrinks every primal step and grows every dual step by the same factor
    ok &= np.allclose(tau1, 0.99 / want_w, rtol=1e-14)
    ok &= np.allclose(eta1, 0.99 / want_y, rtol=1e-14)
    ok &= np.allclose(tau2, 0.5 * tau1, rtol=1e-14) and np.allclose(eta2, 2.0 * eta1, rtol=1e-14)
    return bool(ok)


def test_diagonal_scales_and_steps_hand_built_inner_qp():
    assert _diagonal_pins_hold()


# ---------------------------------------------------------------------------
# row normalisation: upper-bound and two-sided rows
# ---------------------------------------------------------------------------

# each case ends with an upper bound active: on the two-sided row of the
# first, on both upper-bound rows of the second, and so on
GENERAL_CASES = [(("eq", "upper", "two"), 1), (("upper", "upper"), 10), (("upper", "eq"), 5),
                 (("two", "lower"), 4), (("two", "two", "eq"), 1), (("two", "two"), 7)]


def _general_case_matches(kinds, seed, time_limit=20.0):
    p = qpgen.tiny_general_qp(3, seed, kinds)
    res = O.solve(p, O.Settings(eps_abs=1e-9, eps_rel=1e-9, max_outer=3000,
                                time_limit=time_limit))
    if res.status != O.SOLVED:
        return False
    pts = kkt_points_general(p["Q"].toarray(), p["c"], p["A"].toarray(), p["rl"], p["ru"],
                             p["xl"], p["xu"])
    near = [lam for x, lam in pts if np.abs(res.x - x).max() < 1e-6]
    return bool(near) and min(np.abs(res.lam - lam).max() for lam in near) < 1e-6


@pytest.mark.parametrize("kinds,seed", GENERAL_CASES)
def test_general_rows_end_at_enumerated_kkt_point(kinds, seed):
    assert _general_case_matches(kinds, seed)


# ---------------------------------------------------------------------------
# mutation checks: a planted mistake makes a pin fail
# ---------------------------------------------------------------------------

def test_mutation_primal_weight_ratio_flipped(monkeypatch):
    def bad(omega, d_w, d_y):
        if d_w > 0 and d_y > 0:
            return math.exp(0.25 * math.log(d_w / d_y) + 0.75 * math.log(omega))
        return omega
    monkeypatch.setattr(O, "primal_weight_update", bad)
    assert not _weight_pins_hold()


def test_mutation_primal_weight_full_step(monkeypatch):
    def bad(omega, d_w, d_y):
        return d_y / d_w if d_w > 0 and d_y > 0 else omega
    monkeypatch.setattr(O, "primal_weight_update", bad)
    assert not _weight_pins_hold()


def test_mutation_tolerance_factor_bounds_swapped(monkeypatch):
    def bad(x_new, z, gamma, r_d, st):
        d = float(np.max(np.abs(x_new - z)))
        ratio = 1.0 if r_d == 0 else min(1.0, d / gamma / r_d)
        return st.rho_in_min - (st.rho_in_min - st.rho_in_max) * ratio
    monkeypatch.setattr(O, "inner_tolerance_factor", bad)
    assert not _tolerance_factor_pins_hold()


def test_mutation_penalty_trigger_inverted(monkeypatch):
    monkeypatch.setattr(O, "penalty_update", _inverted)
    assert not _penalty_pins_hold()
    rules = _run_rules(qpgen.workload("small", 1), O.Settings(), 25)
    assert not _rules_invariants_hold(rules, O.Settings())


def _inverted(sigma, r_new, r_prev, active, gate_tol, st):
    """Raises the rows whose residual DID fall below 0.25 of the previous one."""
    trig = (np.abs(r_new) < st.theta_sigma * np.abs(r_prev)) & active
    rn = float(np.max(np.abs(r_new))) if r_new.size else 0.0
    if rn <= 0:
        return sigma.copy(), np.zeros_like(trig)
    fac = np.maximum(1.0, st.sigma_growth * np.abs(r_new) / rn)
    return np.where(trig, np.minimum(st.sigma_max, sigma * fac), sigma), trig


def test_mutation_penalty_inactive_rows_raised(monkeypatch):
    orig = O.penalty_update

    def bad(sigma, r_new, r_prev, active, gate_tol, st):
        return orig(sigma, r_new, r_prev, np.ones_like(active), gate_tol, st)
    monkeypatch.setattr(O, "penalty_update", bad)
    assert not _penalty_pins_hold()


def test_mutation_centre_condition_inverted(monkeypatch):
    def bad(x_new, z, r_p, s_p, eps_ak, eps_rk, st, floor=None):
        if r_p > eps_ak + eps_rk * s_p:
            return x_new.copy(), eps_ak * st.rho_z, eps_rk * st.rho_z, True
        return z, eps_ak, eps_rk, False
    monkeypatch.setattr(O, "center_update", bad)
    assert not _centre_pins_hold()


def test_mutation_centre_tolerances_not_shrunk(monkeypatch):
    def bad(x_new, z, r_p, s_p, eps_ak, eps_rk, st, floor=None):
        if r_p <= eps_ak + eps_rk * s_p:
            return x_new.copy(), eps_ak, eps_rk, True
        return z, eps_ak, eps_rk, False
    monkeypatch.setattr(O, "center_update", bad)
    assert not _centre_pins_hold()
    st = O.Settings(penalty_gate=False, center_floor=False)
    assert not _rules_invariants_hold(_run_rules(qpgen.workload("small", 1), st, 25), st)


def test_mutation_penalty_weighted_coupling_dropped(monkeypatch):
    def bad(H, B, sigma, n_xs):
        h1 = np.asarray(abs(H).sum(axis=0)).ravel()
        b1 = np.asarray(abs(B).sum(axis=0)).ravel()
        m_w = h1 + b1
        B2 = B.multiply(B)
        return m_w, np.asarray(B2 @ (1.0 / m_w)).ravel()
    monkeypatch.setattr(O, "diagonal_scales", bad)
    assert not _diagonal_pins_hold()


def test_mutation_primal_weight_placement_swapped(monkeypatch):
    def bad(m_w, m_y, omega, st):
        return 0.99 * omega / m_w, 0.99 / (omega * m_y)
    monkeypatch.setattr(O, "diagonal_steps", bad)
    assert not _diagonal_pins_hold()


def test_mutation_upper_row_not_negated(monkeypatch):
    orig = O.normalise

    def bad(prob):
        P = orig(prob)
        # forget to flip the right-hand side of rows negated from an upper bound
        flip = P.sign_of < 0
        P.b[flip] = -P.b[flip]
        return P
    monkeypatch.setattr(O, "normalise", bad)
    assert not _general_case_matches(("upper", "upper"), 10, time_limit=3.0)


def test_mutation_two_sided_row_upper_side_dropped(monkeypatch):
    orig = O.normalise

    def bad(prob):
        p2 = dict(prob)
        ru = np.array(prob["ru"], float)
        rl = np.array(prob["rl"], float)
        ru[(rl != ru) & np.isfinite(rl)] = np.inf
        p2["ru"] = ru
        return orig(p2)
    monkeypatch.setattr(O, "normalise", bad)
    assert not _general_case_matches(("two", "two", "eq"), 1, time_limit=3.0)


# ---------------------------------------------------------------------------
# tolerance calibration of the experimental protocol (Section 4): a point is
# accepted only when the KKT test on the caller's unscaled problem passes
# ---------------------------------------------------------------------------

def test_calibration_continues_until_unscaled_test_passes():
    """Small seed 2 (Q-aware scaling): the scaled test passes first at a
    point whose unscaled dual residual fails the external test; the internal
    tolerances are halved once and the returned point passes both."""
    p = qpgen.workload("small", 2)
    tr = O.Trace()
    res = O.solve(p, O.Settings(outer_scaling=2, max_outer=5000), trace=tr)
    assert res.status == O.SOLVED and res.halvings == 1
    assert O.passes_external(res, 1e-4, 1e-4)
    k0, ea0, er0, rp0, rd0, sp0, sd0 = tr.external[0]
    assert (ea0, er0) == (1e-4, 1e-4)
    assert rd0 > 1e-4 + 1e-4 * sd0                      # the first candidate fails it
    assert tr.external[-1][1:3] == (5e-5, 5e-5)
    # stopping on the scaled test alone returns that first candidate
    plain = O.solve(p, O.Settings(outer_scaling=2, max_outer=5000, external_halvings=0))
    assert plain.status == O.SOLVED and plain.outer_iters == k0
    assert not O.passes_external(plain, 1e-4, 1e-4)


def test_calibration_limit_reports_inaccurate(monkeypatch):
    """When the external test never passes, the run ends after the allowed
    halvings (1/128 of the requested tolerances) with its own status."""
    orig = O.external_kkt
    calls = []

    def failing(prob, x, lam):
        rp, rd, sp_, sd = orig(prob, x, lam)
        calls.append(1)
        return rp, 1e9, sp_, sd
    monkeypatch.setattr(O, "external_kkt", failing)
    res = O.solve(qpgen.tiny_qp(3, 1, 1, 2), O.Settings(max_outer=20000))
    assert res.status == O.INACCURATE
    assert res.halvings == 7 and len(calls) == 8 + 1   # 8 candidates, then the final report


def test_kkt_pass_limit_ends_the_solve_at_a_check():
    """The KKT pass limit (parameter table, +inf by default): the solve ends
    with MAX_ITER at the first periodic check at which the cumulative trial
    count has reached the limit, and the same run without the limit passes
    that point."""
    prob = qpgen.workload("small", 1)
    tr = O.Trace(max_iters=0)
    res = O.solve(prob, O.Settings(outer_scaling=2, kkt_pass_limit=300), trace=tr)
    assert res.status == O.MAX_ITER
    # checks record (kind, accepted since formation, candidate, trials so far, ratio)
    hit = [c for c in tr.checks if c[0] != "converged" and c[3] >= 300]
    assert hit and tr.checks[-1] is hit[0]
    trials = res.counters.trials
    assert trials == hit[0][3] and 300 <= trials < 300 + 2 * 64
    free = O.solve(prob, O.Settings(outer_scaling=2, max_outer=60))
    assert free.counters.trials > trials
