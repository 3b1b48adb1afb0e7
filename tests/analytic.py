"""Analytic and semi-analytic references used to pin the oracle.

Nothing here is imported by the oracle or by the HIP path; these are
independent statements of what the method must reproduce.
"""
from __future__ import annotations

import math

import numpy as np

SQ3 = math.sqrt(3.0)


# --------------------------------------------------------------------------
# Exact Riemann problem for the conformal gas p = e/3 (Sec. 5.1)
# --------------------------------------------------------------------------

def sod_star_state(eL: float, eR: float):
    """Plateau state (e*, v*) and shock speed for a left rarefaction + right shock.

    Rarefaction: for p = c^2 e the Riemann invariant carried through a
    left-facing fan is artanh(v) + c/(1+c^2) ln e; with c^2 = 1/3 that is
    artanh(v) + (sqrt(3)/4) ln e.  Shock into the resting right state: the
    relative velocity across a relativistic shock obeys
    v^2 = (p2 - p1)(e2 - e1) / ((e1 + p2)(e2 + p1)), and the shock speed is
    [T^{tx}] / [T^{tt}].
    """
    from scipy.optimize import brentq
    pR = eR / 3.0

    def v_raref(e):
        return math.tanh(SQ3 / 4.0 * math.log(eL / e))

    def v_shock(e):
        p = e / 3.0
        return math.sqrt((p - pR) * (e - eR) / ((eR + p) * (e + pR)))

    es = brentq(lambda e: v_raref(e) - v_shock(e), eR * (1 + 1e-12), eL * (1 - 1e-12),
                xtol=1e-15, rtol=1e-15)
    vs = v_raref(es)
    ps = es / 3.0
    w = (es + ps) / (1.0 - vs * vs)
    Vsh = w * vs / (w - ps - eR)
    return es, vs, Vsh


def sod_exact(x, t, eL: float, eR: float):
    """e(x, t), v(x, t) of the Riemann problem with the jump at x = 0, t > 0."""
    c = 1.0 / SQ3
    es, vs, Vsh = sod_star_state(eL, eR)
    xi = np.asarray(x, dtype=np.float64) / t
    tail = (vs - c) / (1.0 - vs * c)
    e = np.empty_like(xi)
    v = np.empty_like(xi)
    left = xi < -c
    fan = (xi >= -c) & (xi < tail)
    star = (xi >= tail) & (xi < Vsh)
    right = xi >= Vsh
    e[left], v[left] = eL, 0.0
    vf = (xi[fan] + c) / (1.0 + xi[fan] * c)
    v[fan] = vf
    e[fan] = eL * np.exp(-4.0 / SQ3 * np.arctanh(vf))
    e[star], v[star] = es, vs
    e[right], v[right] = eR, 0.0
    return e, v


# --------------------------------------------------------------------------
# Bjorken flow ODEs (Secs. 5.4 and 5.5), pi = -tau^2 pi^{eta eta}
# --------------------------------------------------------------------------

def bjorken_rhs(tau, e, pi, Pi, eos_fn, eta_s, zeta_coef, taupipi, zeta_fn=None):
    """Right-hand sides of the 0+1d equations of Secs. 5.4/5.5.

    de/dtau  = -(e + P0 + Pi - pi)/tau
    tau_Pi dPi/dtau + Pi = -zeta/tau - delta_PiPi Pi/tau + lambda_Pipi pi/tau
    tau_pi dpi/dtau + pi = (4/3) eta/tau - (tau_pipi/3 + delta_pipi) pi/tau
                           + (2/3) lambda_piPi Pi/tau
    with the coefficients of Sec. 2.2 (eta = (eta/s) s, s = (e+P0)/T,
    tau_pi = 5 (eta/s)/T, zeta/s = zeta_coef (1/3 - c_s^2), or zeta_coef
    zeta_fn(T) when zeta_fn is given; zeta/tau_Pi = 15 (1/3 - c_s^2)^2 (e+P0)).
    Returned as (de, dpi, dPi); the relaxation equations are divided by their
    times.
    """
    P0, cs2, T = eos_fn(e)
    de = -(e + P0 + Pi - pi) / tau
    dpi = 0.0
    dPi = 0.0
    if eta_s > 0:
        inv_tpi = T / (5.0 * eta_s)
        eta_tpi = (e + P0) / 5.0
        dpi = (4.0 / 3.0) * eta_tpi / tau - pi * inv_tpi - (taupipi / 3.0 + 4.0 / 3.0) * pi / tau \
            + (2.0 / 3.0) * (6.0 / 5.0) * Pi / tau
    if zeta_coef > 0:
        d = 1.0 / 3.0 - cs2
        zeta_tPi = 15.0 * d * d * (e + P0)
        if zeta_fn is None:
            inv_tPi = 15.0 * d * T / zeta_coef
        else:
            inv_tPi = 15.0 * d * d * T / (zeta_coef * zeta_fn(T))
        dPi = -zeta_tPi / tau - Pi * inv_tPi - (2.0 / 3.0) * Pi / tau + (8.0 / 5.0) * d * pi / tau
    return de, dpi, dPi


def bjorken_ode_solution(tau0, tau1, e0, pi0, Pi0, eos_fn, eta_s, zeta_coef, taupipi,
                         t_eval=None, zeta_fn=None):
    from scipy.integrate import solve_ivp

    def f(t, y):
        return list(bjorken_rhs(t, y[0], y[1], y[2], eos_fn, eta_s, zeta_coef, taupipi, zeta_fn))

    sol = solve_ivp(f, (tau0, tau1), [e0, pi0, Pi0], method="DOP853", rtol=1e-12,
                    atol=1e-14, t_eval=t_eval, dense_output=False)
    return sol


def bjorken_reduced_rates(tau, X, eos_fn, eta_s, zeta_coef, taupipi):
    """d/dtau of X = (T^{tau tau}, a = pi^{xx} = pi^{yy}, b = pi^{eta eta}, Pi) for a
    homogeneous state at rest, reduced by hand from the equations of Sec. 2.4
    without assuming tracelessness (an Euler stage keeps 2a + tau^2 b = 0 only to
    O(dtau^2)).  With u = (1,0,0,0): theta = 1/tau, sigma^{xx} = 1/(3 tau),
    sigma^{eta eta} = -2/(3 tau^3), sigma_{xx} = 1/(3 tau), sigma_{eta eta} = -2 tau/3,
    pi:sigma = (2/3)(a/tau - tau b), I_4^{xx} = -a/(3 tau) + (pi:sigma)/3,
    I_4^{eta eta} = 2b/(3 tau) + (pi:sigma)/(3 tau^2), G^{eta eta} = -2b/tau,
    T^{eta eta} = (P0 + Pi)/tau^2 + b."""
    Ttt, a, b, Pi = X
    e = Ttt
    P0, cs2, T = eos_fn(e)
    th = 1.0 / tau
    ps = (2.0 / 3.0) * (a / tau - tau * b)
    dT = -(e + P0 + Pi + tau * tau * b) / tau
    da = db = dPi = 0.0
    if eta_s > 0:
        inv_tpi = T / (5.0 * eta_s)
        eta_tpi = (e + P0) / 5.0
        I4xx = -a / (3 * tau) + ps / 3.0
        I4ee = 2 * b / (3 * tau) + ps / (3 * tau * tau)
        sxx, see = 1.0 / (3 * tau), -2.0 / (3 * tau ** 3)
        da = 2 * eta_tpi * sxx - a * inv_tpi - (4.0 / 3.0) * th * a - taupipi * I4xx + 1.2 * Pi * sxx
        db = (2 * eta_tpi * see - b * inv_tpi - (4.0 / 3.0) * th * b - taupipi * I4ee + 1.2 * Pi * see
              - 2.0 * b / tau)
    if zeta_coef > 0:
        d = 1.0 / 3.0 - cs2
        dPi = -15 * d * d * (e + P0) * th - Pi * 15 * d * T / zeta_coef - (2.0 / 3.0) * Pi * th \
            + 1.6 * d * ps
    return np.array([dT, da, db, dPi])


def bjorken_heun_reduced(tau0, dtau, nsteps, X0, eos_fn, eta_s, zeta_coef, taupipi):
    X = np.array(X0, dtype=np.float64)
    tau = tau0
    for _ in range(nsteps):
        Xs = X + dtau * bjorken_reduced_rates(tau, X, eos_fn, eta_s, zeta_coef, taupipi)
        Xss = Xs + dtau * bjorken_reduced_rates(tau + dtau, Xs, eos_fn, eta_s, zeta_coef, taupipi)
        X = 0.5 * (X + Xss)
        tau += dtau
    return X, tau
