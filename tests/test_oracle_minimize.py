"""Pins of the oracle's minimizer: the curvilinear step (Method section,
eq. (8)), the gradient identities (eq. (2)-(5)), the step rule's invariants,
and the physics it must reproduce (Stoner-Wohlfarth switching, including the
paper's own 45-degree pin, and the Bloch wall).  No GPU."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.fem import ANIS, EXCH, MU0, ZEEM
from oracle.minimize import Options, bisect_switch, cayley, minimize
from paper_1309_5796_amd import meshgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_lagrange_formula_gives_projected_gradient():
    """a x (b x c) = (a.c) b - (a.b) c, so m x (-m x G) = G - (m.G) m for |m| = 1."""
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(size=(3, 50, 3))
    lhs = np.cross(a, np.cross(b, c))
    rhs = np.sum(a * c, 1)[:, None] * b - np.sum(a * b, 1)[:, None] * c
    assert np.abs(lhs - rhs).max() < 1e-13
    m = _unit(rng, 50)
    G = rng.normal(size=(50, 3))
    assert np.abs(np.cross(m, -np.cross(m, G)) - (G - np.sum(m * G, 1)[:, None] * m)).max() < 1e-13


@pytest.mark.parametrize("tau", [1e-6, 0.1, 1.0, 37.0])
def test_cayley_step_solves_implicit_equation_and_keeps_norm(tau):
    rng = np.random.default_rng(1)
    m = _unit(rng, 200)
    h = rng.normal(size=(200, 3)) * 3
    mp = cayley(m, h, tau)
    H = np.cross(m, h)
    resid = mp - m + tau * np.cross(0.5 * (m + mp), H)
    assert np.abs(resid).max() < 1e-13 * max(1.0, tau * np.abs(H).max())
    assert np.abs(np.linalg.norm(mp, axis=1) - 1).max() < 2e-15


def test_cayley_first_order_limit_is_projected_steepest_descent():
    """m+ = m - tau m x H + O(tau^2) = m + tau (h - (m.h) m) + O(tau^2), eq. (6)."""
    rng = np.random.default_rng(2)
    m = _unit(rng, 100)
    h = rng.normal(size=(100, 3))
    errs = []
    for tau in (1e-2, 1e-3):
        lin = m + tau * (h - np.sum(m * h, 1)[:, None] * m)
        errs.append(np.abs(cayley(m, h, tau) - lin).max())
    assert errs[1] < errs[0] / 50


def test_energy_slope_along_the_curve_is_minus_weighted_torque_squared(cfg1, cfg1_system):
    """de/dtau at tau = 0 equals -sum_i V_i |m_i x h_i|^2 (reduced units)."""
    s = cfg1_system
    rng = np.random.default_rng(3)
    m = cfg1["m0"] + 0.2 * rng.normal(size=cfg1["m0"].shape)
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    b = cfg1["b_ext"]
    ev = s.evaluate(m, b)
    H = np.cross(m, ev["h"])
    slope = -float(np.sum(s.V * np.sum(H * H, 1)))
    d = 1e-4 / np.abs(H).max()
    fd = (s.evaluate(cayley(m, ev["h"], d), b)["e"] - s.evaluate(cayley(m, ev["h"], -d), b)["e"]) / (2 * d)
    assert abs(fd - slope) < 1e-6 * abs(slope)


def test_minimize_config1_invariants(cfg1, cfg1_system):
    """Converges below the torque tolerance; |m_i| = 1 after every step; no
    accepted energy exceeds the maximum of the 20 before it."""
    r = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options(record=True))
    assert r.status == 0 and r.max_torque < 1e-6
    assert r.norm_drift < 1e-12
    E = r.energies
    for k in range(1, len(E)):
        assert E[k] <= max(E[max(0, k - 20):k])
    assert E[-1] < E[0]
    assert r.evals >= r.iterations + 1


def _sw_system(psi_deg):
    mesh = meshgen.kuhn_box((1e-9,) * 3, (2, 2, 2), air=False)
    return oracle.System(mesh)


def sw_field(psi):
    """Stoner-Wohlfarth astroid: h_sw = (cos^(2/3) psi + sin^(2/3) psi)^(-3/2) in units of 2 K1 / Ms."""
    return (math.cos(psi) ** (2 / 3) + math.sin(psi) ** (2 / 3)) ** (-1.5)


@pytest.mark.parametrize("psi_deg,tol", [(45.0, 2e-4), (1.0, 2e-4)])
def test_stoner_wohlfarth_switching_field(psi_deg, tol):
    """Small cube, stray field off: uniform rotation, so the switching field is
    the astroid's.  At 45 degrees it is half the anisotropy field, the paper's
    own check of its demagnetization curve (Results, comparison section)."""
    s = _sw_system(psi_deg)
    psi = math.radians(psi_deg)
    u = np.array([math.sin(psi), 0.0, math.cos(psi)])
    mu0HK = 2 * meshgen.K1_JM3 / (meshgen.JS_T / MU0)
    o = Options(terms=EXCH | ANIS | ZEEM, tol=1e-9, max_evals=200000)
    m = np.tile([0.0, 0.0, 1.0], (s.N, 1))
    exact = sw_field(psi) * mu0HK
    # start below the switching field, step past it, then bisect
    B_lo, B_hi = -0.97 * exact * u, -1.03 * exact * u
    r = minimize(s, m, B_lo, o)
    assert s.mean_m(r.m) @ u > 0
    r2 = minimize(s, r.m, B_hi, o)
    assert s.mean_m(r2.m) @ u < 0
    b_sw = -bisect_switch(s, r.m, B_lo, B_hi, u, 1e-4 * mu0HK, o)
    assert abs(b_sw - exact) < tol * exact


def test_paper_pin_45deg_coercive_field_is_half_anisotropy_field():
    with open(os.path.join(GOLDEN, "paper_pins.json")) as f:
        pins = json.load(f)
    assert abs(sw_field(math.radians(45.0)) - pins["coercive_field_over_anisotropy_field_at_45deg"]) < 1e-15


def test_sw_loop_matches_brute_force_single_spin():
    """Hysteresis continuation of the uniform cube vs a brute-force
    continuation of e(theta) = K1 sin^2(theta) - Ms B cos(theta - psi)."""
    s = _sw_system(1.0)
    psi = math.radians(1.0)
    u = meshgen.U_H_1DEG
    Ms = meshgen.JS_T / MU0
    Bs = np.concatenate([np.arange(8.0, -8.01, -0.5), np.arange(-7.5, 8.01, 0.5)])
    recs, _ = oracle.hysteresis(s, np.tile([0.0, 0.0, 1.0], (s.N, 1)), Bs[:, None] * u[None, :],
                                Options(terms=EXCH | ANIS | ZEEM, tol=1e-9))
    theta = 0.0
    grid = np.linspace(-1e-3, 1e-3, 2001)
    for B, rec in zip(Bs, recs):
        # follow the local minimum in theta by steepest descent
        for _ in range(200000):
            g = 2 * meshgen.K1_JM3 * math.sin(theta) * math.cos(theta) + Ms * B * math.sin(theta - psi)
            step = -g / (2 * meshgen.K1_JM3 + 2 * Ms * abs(B)) * 0.5
            theta += step
            if abs(step) < 1e-13:
                break
        e = meshgen.K1_JM3 * np.sin(theta + grid) ** 2 - Ms * B * np.cos(theta + grid - psi)
        assert np.argmin(e) == 1000                   # a true local minimum
        m1 = math.cos(theta - psi)
        assert abs(float(rec.m_avg @ u) - m1) < 1e-6, (B, float(rec.m_avg @ u), m1)


def _bloch(cells_per_nm):
    n = 64 * cells_per_nm
    mesh = meshgen.kuhn_box((32e-9, 0.5e-9, 0.5e-9), (n, cells_per_nm, cells_per_nm), air=False)
    s = oracle.System(mesh)
    x = mesh.xyz[s.nodes, 0]
    d0 = math.sqrt(meshgen.A_JM / meshgen.K1_JM3)
    th = 2 * np.arctan(np.exp(x / d0))
    m = np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], axis=1)
    r = minimize(s, m, np.zeros(3), Options(terms=EXCH | ANIS, tol=1e-8))
    assert r.status == 0
    sigma = r.E / 1e-18
    # for theta = 2 atan(exp(x/d0)), integral of sin^2(theta) dx = 2 d0, so the
    # wall width pi d0 is pi/2 times that integral per unit cross-section
    width = 0.5 * math.pi * float(np.sum(s.V * (1.0 - r.m[:, 2] ** 2))) / 1e-18
    return sigma, width


def test_bloch_wall_energy_and_width_converge_second_order():
    sig_exact = 4 * math.sqrt(meshgen.A_JM * meshgen.K1_JM3)
    w_exact = math.pi * math.sqrt(meshgen.A_JM / meshgen.K1_JM3)
    s1, w1 = _bloch(1)
    s2, w2 = _bloch(2)
    e1, e2 = (s1 - sig_exact) / sig_exact, (s2 - sig_exact) / sig_exact
    assert abs(e1) < 0.04 and abs(e2) < 0.01
    assert 3.0 < e1 / e2 < 6.0                        # O(h^2)
    f1, f2 = (w1 - w_exact) / w_exact, (w2 - w_exact) / w_exact
    assert abs(f1) < 0.10 and abs(f2) < 0.025
    assert 3.0 < f1 / f2 < 6.0                        # O(h^2)


@pytest.mark.parametrize("rule", ["alternate", "bb1", "bb2"])
def test_other_step_rules_reach_the_same_minimum(cfg1, cfg1_system, rule):
    """The paper mentions plain alternation of tau1/tau2 before choosing the
    adaptive rule; every rule must reach the same local minimum."""
    ref = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options())
    r = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options(step_rule=rule, record=True))
    assert r.status == 0 and r.max_torque < 1e-6
    scale = sum(abs(v) for v in ref.terms.values())
    assert abs(r.E - ref.E) < 1e-9 * scale
    E = r.energies
    for k in range(1, len(E)):
        assert E[k] <= max(E[max(0, k - 20):k])


# ---------------------------------------------------------------------------
# Pins of the step-rule decisions (Method section, step length selection,
# eq. (10) and the 20-energy nonmonotone rule).  The constants are the
# readings the library shares with the oracle: first trial 0.1 / max|H|;
# Armijo c1 = 1e-4 with slope -sum V |H|^2, halving; BB trials accepted
# against the maximum of the last 20 accepted energies; adaptive switch with
# kappa0 = 0.5, a window of the last 3 tau2 values, kappa *= 0.9 / 1.1;
# s.y <= 0 gives 10 tau; tau clamped to [1e-10, 1e10].
# ---------------------------------------------------------------------------

def _spin_model(theta0_m, B, psi, th0=0.1, tol=1e-10, M=20, max_evals=1000, c1=1e-4):
    """The same minimizer for one uniformly magnetized spin, written in its
    rotation angle instead of vectors.  m = (sin t, 0, cos t), easy axis z,
    field B (sin psi, 0, cos psi): the reduced energy per volume is
    eps(t) = k sin^2 t - (B / Js) cos(t - psi) with k = K1 / (mu0 Ms^2); the
    torque m x h is -eps'(t) y, the projected gradient g = eps'(t) dm/dt, and
    the Cayley step is the rotation t -> t - 2 atan(tau eps'(t) / 2) about y.
    Volume factors cancel from every ratio and comparison.  Returns the
    trials (tau, accepted) and the step-length decisions."""
    Ms = meshgen.JS_T / MU0
    k = meshgen.K1_JM3 / (MU0 * Ms * Ms)
    beta = B / meshgen.JS_T

    def eps(t):
        return k * math.sin(t) ** 2 - beta * math.cos(t - psi)

    def deps(t):
        return 2 * k * math.sin(t) * math.cos(t) + beta * math.sin(t - psi)

    def mvec(t):
        return np.array([math.sin(t), 0.0, math.cos(t)])

    def gvec(t):
        return deps(t) * np.array([math.cos(t), 0.0, -math.sin(t)])

    t = theta0_m
    hist = [eps(t)]
    T = abs(deps(t))
    trials, steps = [], []
    if T < tol:
        return trials, steps, 1
    tau, kappa, window, first, evals = th0 / T, 0.5, [], True, 1
    while True:
        ref = max(hist[-M:])
        d = deps(t) ** 2
        back = False
        while True:
            tt = t - 2.0 * math.atan(0.5 * tau * deps(t))
            et = eps(tt)
            evals += 1
            ok = et <= ref - c1 * tau * d if (first or back) else et <= ref
            trials.append((tau, ok))
            if ok:
                break
            tau *= 0.5
            back = True
        s = mvec(tt) - mvec(t)
        y = gvec(tt) - gvec(t)
        ss, sy, yy = s @ s, s @ y, y @ y
        t = tt
        hist.append(et)
        if abs(deps(t)) < tol or evals >= max_evals:
            return trials, steps, evals
        first = False
        if sy <= 0:
            tau, branch, t1, t2 = min(10 * tau, 1e10), "grow", None, None
        else:
            t1, t2 = ss / sy, sy / yy
            window = (window + [t2])[-3:]
            if t2 / t1 < kappa:
                tau, branch = min(window), "tau2min"
                kappa *= 0.9
            else:
                tau, branch = t1, "tau1"
                kappa *= 1.1
        tau = min(max(tau, 1e-10), 1e10)
        steps.append(dict(t1=t1, t2=t2, branch=branch, kappa_out=kappa, tau=tau))


@pytest.mark.parametrize("th_m,B,psi_deg,th0,c1", [(0.3, -6.5, 1.0, 0.1, 1e-4), (2.5, -3.0, 10.0, 0.1, 1e-4),
                                                    (2.5, -3.0, 10.0, 3.0, 1e-4), (1.0, 2.0, 60.0, 0.1, 1e-4),
                                                    (2.5, -3.0, 10.0, 3.0, 0.45)],
                         ids=["near-switching", "reversal", "first-trial-rejected", "oblique", "strict-armijo"])
def test_step_decisions_match_single_spin_angle_model(th_m, B, psi_deg, th0, c1):
    """On a uniformly magnetized cube with only the nodal terms (anisotropy
    and Zeeman: no coupling between nodes) every node turns exactly alike, so
    the oracle's vector iteration must reproduce the
    single-spin recurrence in the rotation angle: the same trial step
    lengths, accept/reject verdicts (first-step Armijo, nonmonotone BB
    acceptance, halving), BB values tau1 = s.s/s.y and tau2 = s.y/y.y, the
    branch of the adaptive switch, kappa and the next step length."""
    s = _sw_system(psi_deg)
    psi = math.radians(psi_deg)
    m0 = np.tile([math.sin(th_m), 0.0, math.cos(th_m)], (s.N, 1))
    b = B * np.array([math.sin(psi), 0.0, math.cos(psi)])
    r = minimize(s, m0, b, Options(terms=ANIS | ZEEM, tol=1e-10, theta0=th0, c1=c1, record=True))
    trials, steps, evals = _spin_model(th_m, B, psi, th0=th0, c1=c1)
    assert r.evals == evals and len(r.trials) == len(trials) and len(r.steps) == len(steps)
    for got, (tau, ok) in zip(r.trials, trials):
        assert got["accepted"] == ok
        assert abs(got["tau"] - tau) <= 1e-8 * tau
    for got, want in zip(r.steps, steps):
        assert got["branch"] == want["branch"]
        if want["t1"] is not None:
            assert abs(got["t1"] - want["t1"]) <= 1e-8 * abs(want["t1"])
            assert abs(got["t2"] - want["t2"]) <= 1e-8 * abs(want["t2"])
        assert abs(got["kappa_out"] - want["kappa_out"]) <= 1e-12
        assert abs(got["tau"] - want["tau"]) <= 1e-8 * want["tau"]
    branches = {x["branch"] for x in r.steps}
    if th_m == 0.3:   # this start exercises every branch of the rule
        assert branches == {"tau1", "tau2min", "grow"}
    if c1 > 0.1:      # a trial that decreases the energy but not by Armijo's margin is rejected
        assert any(not x["accepted"] and x["e"] < x["e_ref"] for x in r.trials)


def test_first_trial_rejection_halves_tau_under_armijo():
    """A first trial step of 3 rad overshoots: it is rejected, tau halves,
    and the accepted trial satisfies the Armijo decrease from the initial
    energy while its predecessor did not."""
    s = _sw_system(10.0)
    psi = math.radians(10.0)
    m0 = np.tile([math.sin(2.5), 0.0, math.cos(2.5)], (s.N, 1))
    b = -3.0 * np.array([math.sin(psi), 0.0, math.cos(psi)])
    r = minimize(s, m0, b, Options(terms=EXCH | ANIS | ZEEM, tol=1e-10, theta0=3.0, record=True))
    t0, t1 = r.trials[0], r.trials[1]
    assert t0["armijo"] and not t0["accepted"]
    assert t1["armijo"] and t1["accepted"] and t1["tau"] == 0.5 * t0["tau"]
    assert t0["e"] > t0["e_ref"] - 1e-4 * t0["tau"] * t0["d"]
    assert t1["e"] <= t1["e_ref"] - 1e-4 * t1["tau"] * t1["d"]
    assert t1["e_ref"] == r.energies[0]


@pytest.mark.parametrize("M", [1, 20])
def test_acceptance_replays_against_the_last_M_accepted_energies(cfg1, cfg1_system, M):
    """Replay every recorded trial of the config-1 minimization: its
    reference is the maximum of the last M accepted energies (the current one
    included), the Armijo form applies to the first trial and to every trial
    after a rejection, and the verdict follows from those alone."""
    r = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options(record=True, M=M))
    hist = [r.energies[0]]
    armijo_next = True
    for tr in r.trials:
        ref = max(hist[-M:])
        assert tr["e_ref"] == ref
        assert tr["armijo"] == armijo_next
        want = tr["e"] <= ref - 1e-4 * tr["tau"] * tr["d"] if tr["armijo"] else tr["e"] <= ref
        assert tr["accepted"] == want
        if tr["accepted"]:
            hist.append(tr["e"])
            armijo_next = False
        else:
            armijo_next = True
    assert hist == r.energies
    raises = sum(1 for k in range(1, len(hist)) if hist[k] > hist[k - 1])
    if M == 1:
        assert raises == 0                    # memory 1 is a monotone line search
    else:
        assert raises >= 1                    # the nonmonotone rule accepts energy increases


def test_sum_of_squares_stopping_test(cfg1, cfg1_system):
    """The paper's stopping test (Results: the squared projected gradient
    summed over the nodes below 1e-12) ends a run only when every node's
    torque is below 1e-6 too, and later than the max-torque test."""
    r_max = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options())
    r_sum = minimize(cfg1_system, cfg1["m0"], cfg1["b_ext"], Options(stop="sumsq"))
    H = np.cross(r_sum.m, r_sum.h)
    assert r_sum.status == 0 and float(np.sum(H * H)) < 1e-12
    assert r_sum.max_torque < 1e-6 and r_sum.evals >= r_max.evals
