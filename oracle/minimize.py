"""Curvilinear steepest descent with modified Barzilai-Borwein steps -- oracle
(test infrastructure only; see the package docstring).

Method section of Exl et al.:
* projected gradient g = m x (-m x grad phi) (eq. (2)-(4)); with the effective
  field h = -grad phi (in units of Ms, variational and lumped, see ``fem``)
  this is g_i = m_i x H_i with H_i = m_i x h_i (eq. (5));
* curvilinear step m+ = m - tau (m + m+)/2 x H(m) (eq. (8)), solved exactly
  (it is a Cayley transform, so |m+| = |m|);
* BB step lengths tau1 = s.s / s.y, tau2 = s.y / y.y (eq. (10)) chosen by the
  adaptive rule of Loris et al. 2009; the first step from an inexact line
  search; a line search whenever the new energy exceeds the previous 20
  (end of the step-length subsection);
* hysteresis as the path of successive local minima under field continuation
  (Introduction, Kinderlehrer and Ma).

Readings where the paper gives no constants (all binding on the library too):
first trial tau = 0.1 / max|H|; Armijo c1 = 1e-4 with the directional
derivative -sum V |H|^2 and halving; acceptance of a BB trial when its energy
is <= the maximum of the last 20 accepted energies; kappa_0 = 0.5, window of
the last 3 tau2 values, kappa *= 0.9 / 1.1; s.y <= 0 gives tau <- 10 tau;
tau clamped to [1e-10, 1e10]; backtracking stops below tau = 1e-14.
Inner products are volume-weighted, <x, y>_V = sum_i V_i x_i . y_i.

Pins (tests/test_oracle_minimize.py): the decisions of the step rule -- trial
step lengths, accept/reject verdicts, tau1 and tau2, the branch of the
adaptive switch, kappa -- equal those of an independent single-spin
recurrence written in the rotation angle (a uniformly magnetized cube with
only nodal terms turns as one spin); a strict Armijo constant rejects
trials that lower the energy by less than its margin; every recorded
verdict replays against the last M accepted energies, memory 1 gives a
monotone search and memory 20 accepts energy increases; plus the
invariants (|m| = 1, the energy bound, the stopping test) and the physics
fixtures (Stoner-Wohlfarth, Bloch wall).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .fem import ALL_TERMS

OK, MAXEVALS, FLOOR = 0, 1, 2


@dataclass
class Options:
    tol: float = 1e-6          # stop when max_i |m_i x h_i| < tol (h in units of Ms)
    max_evals: int = 100000
    terms: int = ALL_TERMS
    M: int = 20                # nonmonotone memory
    c1: float = 1e-4
    rho: float = 0.5
    kappa0: float = 0.5
    M_alpha: int = 2           # window of M_alpha + 1 tau2 values
    tau_min: float = 1e-10
    tau_max: float = 1e10
    tau_floor: float = 1e-14
    theta0: float = 0.1
    step_rule: str = "adaptive"  # "adaptive" (the paper's choice), "alternate", "bb1", "bb2"
    stop: str = "max"          # "max": max_i |m_i x h_i| < tol; "sumsq": sum_i |m_i x h_i|^2 < tol^2,
                               # the paper's test on the squared projected gradient (Results)
    record: bool = False       # keep per-step diagnostics


@dataclass
class Result:
    m: np.ndarray
    h: np.ndarray
    e: float
    E: float
    terms: dict
    max_torque: float
    sum_V_torque2: float
    iterations: int
    evals: int
    status: int
    energies: List[float] = field(default_factory=list)
    norm_drift: float = 0.0
    trials: List[dict] = field(default_factory=list)
    steps: List[dict] = field(default_factory=list)


def cross(a, b):
    return np.cross(a, b)


def cayley(m: np.ndarray, h: np.ndarray, tau: float) -> np.ndarray:
    """Exact solution of m+ = m - tau (m + m+)/2 x H with H = m x h.

    Writing a = (tau/2) H, eq. (8) reads (I - [a]x) m+ = (I + [a]x) m, whose
    solution is m+ = m + 2 (c + a x c) / (1 + a.a) with c = a x m (the
    Rodrigues form of the Cayley transform: an exact rotation of m).
    """
    a = 0.5 * tau * cross(m, h)
    c = cross(a, m)
    return m + 2.0 * (c + cross(a, c)) / (1.0 + np.sum(a * a, axis=1, keepdims=True))[:, :]


def _vdot(V, x, y):
    return float(np.sum(V[:, None] * x * y))


def minimize(sys, m0: np.ndarray, b_ext, opts: Optional[Options] = None) -> Result:
    """Algorithm of the Method section on the sphere; returns the local minimum
    reached from m0 at applied field b_ext (T)."""
    o = opts or Options()
    V = sys.V
    m = np.array(m0, dtype=float)
    nrm = np.linalg.norm(m, axis=1)
    if np.any(nrm == 0):
        raise ValueError("zero magnetization vector")
    m /= nrm[:, None]

    ev = sys.evaluate(m, b_ext, o.terms)
    evals = 1
    h, e = ev["h"], ev["e"]
    H = cross(m, h)
    Tn = np.linalg.norm(H, axis=1)
    T = float(Tn.max())

    def converged(H_):
        if o.stop == "sumsq":
            return float(np.sum(H_ * H_)) < o.tol * o.tol
        return float(np.linalg.norm(H_, axis=1).max()) < o.tol

    hist = [e]
    drift = 0.0
    # with record=True: every trial (tau, its energy, the reference it was
    # tested against, whether the Armijo form applied, the verdict) and every
    # step-length decision after an accepted step
    trials: List[dict] = []
    steps: List[dict] = []

    def result(status, iters):
        return Result(m=m, h=h, e=e, E=ev["E"], terms={k: ev[k] for k in ("E_ex", "E_an", "E_Z", "E_d")},
                      max_torque=T, sum_V_torque2=float(np.sum(V * np.sum(H * H, axis=1))),
                      iterations=iters, evals=evals, status=status,
                      energies=list(hist) if o.record else [], norm_drift=drift,
                      trials=trials, steps=steps)

    if converged(H):
        return result(OK, 0)
    tau = o.theta0 / T
    kappa = o.kappa0
    window: List[float] = []
    alt = False
    first = True
    iters = 0
    while True:
        e_ref = max(hist[-o.M:])
        d = float(np.sum(V * np.sum(H * H, axis=1)))
        backtrack = False
        while True:
            m_t = cayley(m, h, tau)
            ev_t = sys.evaluate(m_t, b_ext, o.terms)
            evals += 1
            e_t = ev_t["e"]
            armijo = first or backtrack
            if armijo:
                ok = e_t <= e_ref - o.c1 * tau * d
            else:
                ok = e_t <= e_ref
            if o.record:
                trials.append(dict(tau=tau, e=e_t, e_ref=e_ref, d=d, armijo=armijo, accepted=ok))
            if ok:
                break
            if evals >= o.max_evals:
                return result(MAXEVALS, iters)
            tau *= o.rho
            backtrack = True
            if tau < o.tau_floor:
                return result(FLOOR, iters)
        h_t = ev_t["h"]
        H_t = cross(m_t, h_t)
        s = m_t - m
        y = cross(m_t, H_t) - cross(m, H)          # g = m x H
        ss, sy, yy = _vdot(V, s, s), _vdot(V, s, y), _vdot(V, y, y)
        drift = max(drift, float(np.abs(np.linalg.norm(m_t, axis=1) - 1.0).max()))
        m, h, e, H, ev = m_t, h_t, e_t, H_t, ev_t
        hist.append(e)
        iters += 1
        T = float(np.linalg.norm(H, axis=1).max())
        if converged(H):
            return result(OK, iters)
        if evals >= o.max_evals:
            return result(MAXEVALS, iters)
        first = False
        rec = dict(ss=ss, sy=sy, yy=yy, kappa_in=kappa, branch="grow")
        if sy <= 0.0:
            tau = min(10.0 * tau, o.tau_max)
        else:
            t1, t2 = ss / sy, sy / yy
            rec["branch"] = o.step_rule
            if o.step_rule == "bb1":
                tau = t1
            elif o.step_rule == "bb2":
                tau = t2
            elif o.step_rule == "alternate":
                # plain alternation, starting with tau1 (step-length subsection)
                tau = t2 if alt else t1
                alt = not alt
            else:
                window.append(t2)
                window = window[-(o.M_alpha + 1):]
                if t2 / t1 < kappa:
                    tau = min(window)
                    kappa *= 0.9
                    rec["branch"] = "tau2min"
                else:
                    tau = t1
                    kappa *= 1.1
                    rec["branch"] = "tau1"
            rec.update(t1=t1, t2=t2)
        tau = min(max(tau, o.tau_min), o.tau_max)
        if o.record:
            rec.update(kappa_out=kappa, tau=tau)
            steps.append(rec)


@dataclass
class StepRecord:
    b: np.ndarray
    m_avg: np.ndarray
    e: float
    E: float
    evals: int
    iterations: int
    status: int
    max_torque: float


def hysteresis(sys, m0: np.ndarray, fields: np.ndarray, opts: Optional[Options] = None):
    """Continuation of local minima along the field list (Introduction,
    Hysteresis): each point starts from the previous minimum with a fresh
    step-length state.  Returns (records, final m)."""
    m = np.array(m0, float)
    recs = []
    for B in np.asarray(fields, float):
        r = minimize(sys, m, B, opts)
        m = r.m
        recs.append(StepRecord(B.copy(), sys.mean_m(m), r.e, r.E, r.evals, r.iterations,
                               r.status, r.max_torque))
    return recs, m


def switching_fields(records, u_hat) -> List[int]:
    """Indices k where sign(<m>.u_hat) differs from the sign at k-1."""
    s = np.sign([float(r.m_avg @ u_hat) for r in records])
    return [k for k in range(1, len(s)) if s[k] != s[k - 1]]


def bisect_switch(sys, m_before: np.ndarray, B_lo, B_hi, u_hat, tol_T: float,
                  opts: Optional[Options] = None) -> float:
    """Switching field between B_lo (unswitched, minimum m_before) and B_hi
    (switched): bisect the segment until it is shorter than tol_T, restarting
    each trial from the last unswitched minimum.  Returns the midpoint of the
    final bracket projected on u_hat (T)."""
    B_lo, B_hi = np.asarray(B_lo, float), np.asarray(B_hi, float)
    s0 = np.sign(float(sys.mean_m(m_before) @ u_hat))
    m_lo = np.array(m_before)
    while np.linalg.norm(B_hi - B_lo) > tol_T:
        mid = 0.5 * (B_lo + B_hi)
        r = minimize(sys, m_lo, mid, opts)
        if np.sign(float(sys.mean_m(r.m) @ u_hat)) != s0:
            B_hi = mid
        else:
            B_lo, m_lo = mid, r.m
    return float(0.5 * (B_lo + B_hi) @ u_hat)
