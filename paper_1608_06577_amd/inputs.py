"""Seeded synthetic inputs: equation-of-state tables and initial primitive fields.

This module is shared by the HIP path's callers and by the oracle's tests.  It
holds none of the arithmetic of the hydrodynamic method itself (no
reconstruction, flux, source term, inversion, regulator or time step): it only
produces

* equation-of-state tables p(e), c_s^2(e), T(e) on ln-uniform e grids, and
* initial primitive fields (e, u^mu, pi^{mu nu}, Pi) on a cell-centred grid.

Units are fm-based natural units throughout: e and p in fm^-4, T in fm^-1,
tau in fm/c, x and y in fm, eta_s dimensionless.  Energy densities quoted in
GeV/fm^3 are converted with hbar*c.

Array layout: every field is component-first, ``(ncomp, neta, ny, nx)``, with
x fastest and eta slowest (the memory order of Sec. 4.2 of the paper).
Component orders:

* u:  (u^tau, u^x, u^y, u^eta)
* pi: (tt, tx, ty, te, xx, xy, xe, yy, ye, ee)  -- the ordering of the
  dissipative state vector in Sec. 3.1 (vector ``pi`` of Eq. qComponents).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HBARC = 0.1973269804  # GeV fm

#: Stefan-Boltzmann constant of a massless gas with 16 degrees of freedom,
#: e = (16 pi^2 / 30) T^4 (the conformal EOS of the viscous Gubser workload).
A_SB16 = 16.0 * math.pi ** 2 / 30.0

PI_NAMES = ("tt", "tx", "ty", "te", "xx", "xy", "xe", "yy", "ye", "ee")
_PI_INDEX = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (0, 3): 3, (1, 1): 4, (1, 2): 5,
             (1, 3): 6, (2, 2): 7, (2, 3): 8, (3, 3): 9}


def pi_component(mu: int, nu: int) -> int:
    """Index of pi^{mu nu} in the 10-component symmetric storage."""
    return _PI_INDEX[(min(mu, nu), max(mu, nu))]


def gev_fm3_to_fm4(e_gev):
    return np.asarray(e_gev) / HBARC


# --------------------------------------------------------------------------
# Equations of state
# --------------------------------------------------------------------------

@dataclass
class EOS:
    """Either conformal (p = e/3, T = (e/a)^{1/4}) or a table on ln-uniform e.

    For a table, node i sits at ln e_i = ln_e0 + i*dln_e and holds p_i, cs2_i
    and T_i.  Interpolation between nodes is the consumer's business.
    """
    conformal: bool
    a_sb: float = A_SB16
    ln_e0: float = 0.0
    dln_e: float = 0.0
    p: np.ndarray | None = None
    cs2: np.ndarray | None = None
    T: np.ndarray | None = None

    @property
    def n(self) -> int:
        return 0 if self.conformal else int(self.p.shape[0])

    def e_nodes(self) -> np.ndarray:
        return np.exp(self.ln_e0 + self.dln_e * np.arange(self.n))


def eos_conformal(a_sb: float = A_SB16) -> EOS:
    return EOS(conformal=True, a_sb=a_sb)


def _c1_log_p_over_e_deficit(y):
    """ln of (1/3 - p/e) for the synthetic EOS, y = ln(e / 1 GeV fm^-3)."""
    from scipy.special import log_ndtr
    return math.log(0.15 * math.sqrt(2.0 * math.pi)) + 0.5 - y + log_ndtr(y - 1.0)


def c1_cs2(e_fm4):
    """c_s^2(e) = 1/3 - 0.15 exp(-ln^2(e / 1 GeV fm^-3) / 2)."""
    y = np.log(np.asarray(e_fm4) * HBARC)
    return 1.0 / 3.0 - 0.15 * np.exp(-0.5 * y * y)


def c1_pressure(e_fm4):
    """Closed form p(e) = int_0^e c_s^2 de' for the synthetic EOS (fm^-4).

    With y = ln(e/e1), e1 = 1 GeV/fm^3:
    p = e/3 - 0.15 e1 sqrt(2 pi) exp(1/2) Phi(y - 1).
    """
    e = np.asarray(e_fm4, dtype=np.float64)
    y = np.log(e * HBARC)
    return e * (1.0 / 3.0 - np.exp(_c1_log_p_over_e_deficit(y)))


def c1_temperature(e_fm4, a_sb: float = A_SB16):
    """T(e) from d ln T = c_s^2 de / (e + p), normalised to (e/a)^{1/4} as e -> 0.

    Writing g = ln T - ln (e/a)/4 and x = ln e, dg/dx = c_s^2 e/(e+p) - 1/4,
    which vanishes (faster than exponentially) as x -> -inf; g is integrated
    from far below the table with a high-order adaptive integrator.
    """
    from scipy.integrate import solve_ivp
    e = np.atleast_1d(np.asarray(e_fm4, dtype=np.float64))
    x_eval = np.log(e)
    order = np.argsort(x_eval)
    xs = x_eval[order]

    def rhs(x, g):
        ee = math.exp(x)
        y = x + math.log(HBARC)
        cs2 = 1.0 / 3.0 - 0.15 * math.exp(-0.5 * y * y)
        p_over_e = 1.0 / 3.0 - math.exp(_c1_log_p_over_e_deficit(y))
        del ee
        return [cs2 / (1.0 + p_over_e) - 0.25]

    x_start = math.log(1e-30 / HBARC)  # ln(e/e1) = -69: integrand is 0 to double precision
    sol = solve_ivp(rhs, (x_start, xs[-1]), [0.0], method="DOP853",
                    t_eval=xs, rtol=1e-13, atol=1e-16)
    g = np.empty_like(xs)
    g[:] = sol.y[0]
    out = np.empty_like(e)
    out[order] = np.exp(0.25 * (xs - math.log(a_sb)) + g)
    return out.reshape(np.shape(e_fm4)) if np.ndim(e_fm4) else out[0]


def eos_c1_table(n: int = 4096, e_min_gev: float = 1e-7, e_max_gev: float = 1e3,
                 a_sb: float = A_SB16) -> EOS:
    """Non-conformal synthetic EOS table on n ln-uniform points in [e_min, e_max]."""
    ln_e0 = math.log(e_min_gev / HBARC)
    ln_e1 = math.log(e_max_gev / HBARC)
    dln = (ln_e1 - ln_e0) / (n - 1)
    e = np.exp(ln_e0 + dln * np.arange(n))
    return EOS(conformal=False, a_sb=a_sb, ln_e0=ln_e0, dln_e=dln,
               p=c1_pressure(e), cs2=c1_cs2(e), T=c1_temperature(e, a_sb))


def eos_conformal_table(n: int = 4096, e_min: float = 1e-6, e_max: float = 1e4,
                        a_sb: float = A_SB16) -> EOS:
    """The conformal EOS written as a table (exercises the table path)."""
    ln_e0 = math.log(e_min)
    dln = (math.log(e_max) - ln_e0) / (n - 1)
    e = np.exp(ln_e0 + dln * np.arange(n))
    return EOS(conformal=False, a_sb=a_sb, ln_e0=ln_e0, dln_e=dln,
               p=e / 3.0, cs2=np.full(n, 1.0 / 3.0), T=(e / a_sb) ** 0.25)


#: 2+1-flavour lattice-QCD trace anomaly I/T^4 (Wuppertal-Budapest fit of
#: Sec. 2, Eq. traceAnomaly, with the small alpha > 0 that makes the pressure
#: approach the Stefan-Boltzmann limit), t = T / 0.2 GeV
WB_FIT = dict(h0=0.1396, h1=-0.1800, h2=0.0350, f0=2.76, f1=6.79, f2=-5.29, g1=-0.47, g2=1.04,
              alpha=0.01)

#: Stefan-Boltzmann e = a T^4 of massless quarks and gluons, N_c = 3, N_f = 3 (Sec. 2)
A_SB_QCD = 3.0 * (2.0 * (3 ** 2 - 1) + 3.5 * 3 * 3) * math.pi ** 2 / 90.0


def wb_trace_anomaly(T_gev, h1_sign: float = -1.0):
    """I(T)/T^4 of the fit (also for complex T, which the derivative uses).

    The exponential factor is exp(h1_sign h1 / t - h2 / t^2).  The equation as
    printed has h1_sign = +1; with h1 = -0.18 that caps p/T^4 at 0.63 of the
    Stefan-Boltzmann value, against a text that has the pressure approach it.
    The default -1 (the cited fit's form) gives 0.87 and a trace-anomaly peak
    of 4.1 near T = 0.2 GeV.
    """
    f = WB_FIT
    t = np.asarray(T_gev) / 0.2
    core = (f["h0"] / (1.0 + f["alpha"] * t * t)
            + f["f0"] * (np.tanh(f["f1"] * t + f["f2"]) + 1.0) / (1.0 + f["g1"] * t + f["g2"] * t * t))
    return core * np.exp(h1_sign * f["h1"] / t - f["h2"] / (t * t))


def eos_lattice_table(n: int = 4096, e_min_gev: float = 1e-7, e_max_gev: float = 1e3,
                      h1_sign: float = -1.0) -> EOS:
    """The lattice-QCD EOS (Sec. 2, equation of state for nuclear collisions)
    as a table on n ln-uniform points of e in [e_min, e_max] GeV/fm^3
    (h1_sign: see wb_trace_anomaly).

    With P = p/T^4 and phi = I/T^4, dP/d ln T = phi (P vanishes as T -> 0,
    where phi falls like exp(-h2 / t^2)); e = 3p + I; T(e_i) is the root of
    ln e(T) = ln e_i; c_s^2 = dp/de = s / (de/dT), s = (e + p)/T and
    de/dT = 3 s + dI/dT.  Units: e, p in fm^-4, T in fm^-1.
    """
    from scipy.integrate import solve_ivp
    from scipy.optimize import brentq
    lnT0, lnT1 = math.log(0.004), math.log(20.0)        # GeV; P(4 MeV) < 1e-40
    sol = solve_ivp(lambda x, P: [float(wb_trace_anomaly(math.exp(x), h1_sign))], (lnT0, lnT1), [0.0],
                    method="DOP853", rtol=1e-13, atol=1e-300, dense_output=True)

    def P(lnT):
        return float(sol.sol(lnT)[0])

    def ln_e_gev4(lnT):
        T = math.exp(lnT)
        return 4.0 * lnT + math.log(3.0 * P(lnT) + float(wb_trace_anomaly(T, h1_sign)))

    ln_e0 = math.log(e_min_gev / HBARC)
    dln = (math.log(e_max_gev / HBARC) - ln_e0) / (n - 1)
    ln_nodes = ln_e0 + dln * np.arange(n) + 4.0 * math.log(HBARC)    # ln e in GeV^4
    # bracket each node on a grid of ln T, then solve
    grid = np.linspace(math.log(0.006), lnT1, 4001)
    lne_grid = np.array([ln_e_gev4(x) for x in grid])
    if not np.all(np.diff(lne_grid) > 0.0):
        raise ValueError("e(T) of the lattice fit is not increasing on the table's range")
    if not (lne_grid[0] < ln_nodes[0] and ln_nodes[-1] < lne_grid[-1]):
        raise ValueError("table range outside the temperatures covered")
    k = np.searchsorted(lne_grid, ln_nodes)
    T = np.empty(n)
    p = np.empty(n)
    cs2 = np.empty(n)
    h = 1e-30
    for i in range(n):
        lnT = brentq(lambda x: ln_e_gev4(x) - ln_nodes[i], grid[k[i] - 1], grid[k[i]], xtol=1e-15, rtol=1e-15)
        Tg = math.exp(lnT)
        phi = float(wb_trace_anomaly(Tg, h1_sign))
        dphi_dT = float(np.imag(wb_trace_anomaly(Tg + 1j * h, h1_sign)) / h)    # complex-step derivative
        pg = P(lnT) * Tg ** 4
        eg = 3.0 * pg + phi * Tg ** 4
        s_ = (eg + pg) / Tg
        dI_dT = 4.0 * Tg ** 3 * phi + Tg ** 4 * dphi_dT
        T[i] = Tg / HBARC
        p[i] = pg / HBARC ** 4
        cs2[i] = s_ / (3.0 * s_ + dI_dT)
    return EOS(conformal=False, a_sb=A_SB_QCD, ln_e0=ln_e0, dln_e=dln, p=p, cs2=cs2, T=T)


# --------------------------------------------------------------------------
# Grids and primitive containers
# --------------------------------------------------------------------------

@dataclass
class Grid:
    nx: int
    ny: int
    neta: int
    dx: float
    dy: float
    deta: float

    @property
    def shape(self):
        return (self.neta, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.neta

    def coords(self):
        """Cell-centre coordinates, each of shape (neta, ny, nx), grid centred at 0."""
        x = (np.arange(self.nx) - 0.5 * (self.nx - 1)) * self.dx
        y = (np.arange(self.ny) - 0.5 * (self.ny - 1)) * self.dy
        h = (np.arange(self.neta) - 0.5 * (self.neta - 1)) * self.deta
        H, Y, X = np.meshgrid(h, y, x, indexing="ij")
        return X, Y, H


@dataclass
class Primitives:
    """Initial primitive fields on a grid (component-first, x fastest)."""
    grid: Grid
    tau0: float
    e: np.ndarray                 # (neta, ny, nx)
    u: np.ndarray                 # (4, neta, ny, nx) contravariant
    pi: np.ndarray                # (10, neta, ny, nx) contravariant
    Pi: np.ndarray                # (neta, ny, nx)
    meta: dict = field(default_factory=dict)


def _zeros_prims(grid: Grid, tau0: float) -> Primitives:
    s = grid.shape
    u = np.zeros((4,) + s)
    u[0] = 1.0
    return Primitives(grid, tau0, np.zeros(s), u, np.zeros((10,) + s), np.zeros(s))


def _metric_diag(tau: float, cartesian: bool):
    g_lo = np.array([1.0, -1.0, -1.0, -1.0 if cartesian else -tau * tau])
    return g_lo, 1.0 / g_lo


# --------------------------------------------------------------------------
# Gubser flow (Sec. 5.6 closed form; Sec. 5.7 viscous, conformal, tau_pipi = 0)
# --------------------------------------------------------------------------

def gubser_rho(tau, r, q):
    """de Sitter time rho(tau, r): sinh rho = -(1 - q^2 tau^2 + q^2 r^2) / (2 q tau)."""
    return -np.arcsinh((1.0 - q * q * tau * tau + q * q * r * r) / (2.0 * q * tau))


def gubser_kappa(tau, r, q):
    """Transverse rapidity of Gubser flow, Sec. 5.6."""
    return np.arctanh(2.0 * q * q * tau * r / (1.0 + q * q * tau * tau + q * q * r * r))


def gubser_ideal_T(tau, r, q, T0hat):
    """Ideal Gubser temperature, closed form of Sec. 5.6 (fm^-1)."""
    br = 1.0 + 2.0 * q * q * (tau * tau + r * r) + q ** 4 * (tau * tau - r * r) ** 2
    return T0hat * (2.0 * q * tau) ** (2.0 / 3.0) / (tau * br ** (1.0 / 3.0))


def gubser_viscous_ode(rho_eval, rho0, That0, eta_s):
    """Conformal Israel-Stewart Gubser flow with tau_pipi = 0 (Sec. 5.7).

    In the Weyl-rescaled de Sitter frame the fluid is static and, with
    pibar = pihat^{eta eta} / (ehat + phat) and tau_pi = 5 (eta/s) / T,
      dT/drho     = T (-2/3 + pibar/3) tanh rho
      dpibar/drho = (4/15) tanh rho - (4/3) pibar^2 tanh rho - pibar T / (5 eta/s)
    (derivation: energy equation D e + (e+P) theta - pi:sigma = 0 and the
    shear relaxation equation of Sec. 2.2 with theta = 2 tanh rho and
    sigma^eta_eta = -(2/3) tanh rho).  Integrated both ways from rho0 with
    T(rho0) = That0, pibar(rho0) = 0.  Returns (That(rho), pibar(rho)).
    """
    from scipy.integrate import solve_ivp
    rho_eval = np.asarray(rho_eval, dtype=np.float64)
    flat = rho_eval.ravel()

    def rhs(rho, y):
        T, pb = y
        th = math.tanh(rho)
        dT = T * (-2.0 / 3.0 + pb / 3.0) * th
        dp = (4.0 / 15.0) * th - (4.0 / 3.0) * pb * pb * th
        if eta_s > 0:
            dp -= pb * T / (5.0 * eta_s)
        return [dT, dp]

    T_out = np.empty_like(flat)
    p_out = np.empty_like(flat)
    for sel, lim in ((flat >= rho0, flat.max(initial=rho0)), (flat < rho0, flat.min(initial=rho0))):
        if not np.any(sel):
            continue
        pts = np.unique(flat[sel])
        if lim == rho0:
            T_out[sel] = That0
            p_out[sel] = 0.0
            continue
        order = pts if lim > rho0 else pts[::-1]
        sol = solve_ivp(rhs, (rho0, lim), [That0, 0.0], method="DOP853",
                        t_eval=order, rtol=1e-12, atol=1e-14)
        Tm = dict(zip(order, sol.y[0]))
        Pm = dict(zip(order, sol.y[1]))
        T_out[sel] = [Tm[v] for v in flat[sel]]
        p_out[sel] = [Pm[v] for v in flat[sel]]
    return T_out.reshape(rho_eval.shape), p_out.reshape(rho_eval.shape)


def gubser_fields(grid: Grid, tau: float, q: float = 1.0, T0hat: float = 1.2,
                  a_sb: float = A_SB16, eta_s: float = 0.0, tau0: float = 1.0):
    """Gubser-flow primitives at proper time tau on the grid (boost invariant).

    eta_s == 0: ideal closed form.  eta_s > 0: semi-analytic solution whose
    ODE starts at rho0 = rho(tau0, r=0) with the ideal central temperature and
    zero shear stress.  pi^{mu nu} = pi^eta_eta [-(3/2) z^mu z^nu - (1/2) Delta^{mu nu}]
    with z = (0,0,0,1/tau) and pi^eta_eta = -pibar (e + P), the form fixed by
    the flow's symmetry (traceless, transverse, axially symmetric about eta).
    """
    X, Y, _ = grid.coords()
    r = np.sqrt(X * X + Y * Y)
    kap = gubser_kappa(tau, r, q)
    rho = gubser_rho(tau, r, q)
    if eta_s > 0:
        rho0 = float(gubser_rho(tau0, 0.0, q))
        That0 = float(gubser_ideal_T(tau0, 0.0, q, T0hat)) * tau0
        That, pibar = gubser_viscous_ode(rho, rho0, That0, eta_s)
        T = That / tau
    else:
        T = gubser_ideal_T(tau, r, q, T0hat)
        pibar = np.zeros_like(T)
    pr = _zeros_prims(grid, tau)
    pr.e[:] = a_sb * T ** 4
    sk = np.sinh(kap)
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(r > 0, X / r, 0.0)
        cy = np.where(r > 0, Y / r, 0.0)
    pr.u[0] = np.cosh(kap)
    pr.u[1] = cx * sk
    pr.u[2] = cy * sk
    pr.u[3] = 0.0
    if eta_s > 0:
        _, g_hi = _metric_diag(tau, False)
        wmix = -pibar * (4.0 / 3.0) * pr.e      # pi^eta_eta (mixed), e + P = 4e/3
        z = np.array([0.0, 0.0, 0.0, 1.0 / tau])
        for mu in range(4):
            for nu in range(mu, 4):
                delta = (g_hi[mu] if mu == nu else 0.0) - pr.u[mu] * pr.u[nu]
                pr.pi[pi_component(mu, nu)] = wmix * (-1.5 * z[mu] * z[nu] - 0.5 * delta)
    pr.meta.update(kind="gubser", q=q, T0hat=T0hat, eta_s=eta_s, tau0=tau0)
    return pr


# --------------------------------------------------------------------------
# Bjorken flow (Secs. 5.4, 5.5): homogeneous, u = (1,0,0,0)
# --------------------------------------------------------------------------

def bjorken_fields(grid: Grid, tau0: float, e0: float, T0: float, eta_s: float,
                   P0: float, navier_stokes: bool = True, Pi0: float = 0.0):
    """Homogeneous Bjorken state; pi = -tau^2 pi^{eta eta} set to its
    Navier-Stokes value (4/3) eta / tau0 with eta = (eta/s)(e+P)/T when asked."""
    pr = _zeros_prims(grid, tau0)
    pr.e[:] = e0
    pr.Pi[:] = Pi0
    if navier_stokes and eta_s > 0:
        eta = eta_s * (e0 + P0) / T0
        pil = (4.0 / 3.0) * eta / tau0
        pr.pi[pi_component(1, 1)] = 0.5 * pil
        pr.pi[pi_component(2, 2)] = 0.5 * pil
        pr.pi[pi_component(3, 3)] = -pil / (tau0 * tau0)
    pr.meta.update(kind="bjorken", eta_s=eta_s)
    return pr


# --------------------------------------------------------------------------
# Riemann problems in Cartesian coordinates (Secs. 5.1-5.3)
# --------------------------------------------------------------------------

SOD_E_LEFT_GEV = 0.0246
SOD_E_RIGHT_GEV = 0.0015


def sod_fields(grid: Grid, t0: float = 0.0, diagonal: bool = False, axis: int = 0,
               e_left_gev: float = SOD_E_LEFT_GEV, e_right_gev: float = SOD_E_RIGHT_GEV):
    """Fluid at rest with a pressure jump at x = 0 (or along y = x)."""
    X, Y, H = grid.coords()
    coord = (X - Y) / math.sqrt(2.0) if diagonal else (X, Y, H)[axis]
    pr = _zeros_prims(grid, t0)
    pr.e[:] = np.where(coord <= 0.0, e_left_gev, e_right_gev) / HBARC
    pr.meta.update(kind="sod", diagonal=diagonal, axis=axis)
    return pr


def cylinder_fields(grid: Grid, t0: float = 0.0, radius: float = 1.0,
                    e_in_gev: float = SOD_E_LEFT_GEV, e_out_gev: float = SOD_E_RIGHT_GEV):
    X, Y, _ = grid.coords()
    pr = _zeros_prims(grid, t0)
    pr.e[:] = np.where(X * X + Y * Y <= radius * radius, e_in_gev, e_out_gev) / HBARC
    pr.meta.update(kind="cylinder", radius=radius)
    return pr


# --------------------------------------------------------------------------
# Synthetic fluctuating event: Gaussian hot spots at Woods-Saxon positions
# --------------------------------------------------------------------------

def woods_saxon_points(rng: np.random.Generator, n: int, R: float = 6.62,
                       a: float = 0.546) -> np.ndarray:
    """n points from a 3D Woods-Saxon density by radial rejection, isotropic angles."""
    rmax = R + 12.0 * a
    out = []
    while len(out) < n:
        r = rng.uniform(0.0, rmax)
        w = (r / rmax) ** 2 / (1.0 + math.exp((r - R) / a))
        if rng.uniform() < w:
            ct = rng.uniform(-1.0, 1.0)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            st = math.sqrt(max(0.0, 1.0 - ct * ct))
            out.append((r * st * math.cos(ph), r * st * math.sin(ph)))
    return np.array(out)


def hotspot_event(grid: Grid, tau0: float = 0.5, n_hot: int = 200, seed: int = 1,
                  sigma: float = 0.5, R: float = 6.62, a_ws: float = 0.546,
                  e_peak_gev: float = 30.0, eta_flat: float = 2.0, sigma_eta: float = 0.5,
                  e_floor_gev: float = 1e-7) -> Primitives:
    """Transverse profile: sum of Gaussian hot spots (width sigma) centred on
    projected Woods-Saxon positions, scaled so the grid maximum is e_peak;
    longitudinal plateau |eta_s| < eta_flat with Gaussian tails (the factorised
    form of Sec. 6.1); floored at e_floor.  u = (1,0,0,0), pi = Pi = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = woods_saxon_points(rng, n_hot, R, a_ws)
    x = (np.arange(grid.nx) - 0.5 * (grid.nx - 1)) * grid.dx
    y = (np.arange(grid.ny) - 0.5 * (grid.ny - 1)) * grid.dy
    h = (np.arange(grid.neta) - 0.5 * (grid.neta - 1)) * grid.deta
    gx = np.exp(-((x[None, :] - pts[:, 0:1]) ** 2) / (2 * sigma * sigma))   # (n, nx)
    gy = np.exp(-((y[None, :] - pts[:, 1:2]) ** 2) / (2 * sigma * sigma))   # (n, ny)
    eperp = gy.T @ gx                                                       # (ny, nx)
    eperp *= (e_peak_gev / HBARC) / eperp.max()
    ah = np.abs(h)
    eL = np.where(ah < eta_flat, 1.0, np.exp(-((ah - eta_flat) ** 2) / (2 * sigma_eta ** 2)))
    pr = _zeros_prims(grid, tau0)
    pr.e[:] = np.maximum(eL[:, None, None] * eperp[None, :, :], e_floor_gev / HBARC)
    pr.meta.update(kind="hotspot", seed=seed, n_hot=n_hot, points=pts)
    return pr


# --------------------------------------------------------------------------
# Smooth random states (parity and conservation tests)
# --------------------------------------------------------------------------

def random_smooth_fields(grid: Grid, tau: float, seed: int, cartesian: bool = False,
                         e_mean: float = 10.0, e_amp: float = 0.3, u_amp: float = 0.3,
                         ueta_amp: float = 0.1, pi_rel: float = 0.05, Pi_rel: float = 0.02,
                         n_modes: int = 3) -> Primitives:
    """Periodic smooth random fields built from a few low Fourier modes.

    pi^{mu nu} is the transverse traceless projection of a random symmetric
    tensor, so the constraints of Sec. 2.4 hold at t = tau.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = (grid.nx, grid.ny, grid.neta)
    i = np.arange(grid.nx)[None, None, :] / grid.nx
    j = np.arange(grid.ny)[None, :, None] / grid.ny
    k = np.arange(grid.neta)[:, None, None] / grid.neta

    def field_():
        f = np.zeros(grid.shape)
        for _ in range(n_modes):
            kx, ky, kz = (int(rng.integers(0, 3)) if m > 1 else 0 for m in n)
            ph = rng.uniform(0, 2 * math.pi)
            f += rng.normal() * np.cos(2 * math.pi * (kx * i + ky * j + kz * k) + ph)
        return f / math.sqrt(n_modes)

    g_lo, g_hi = _metric_diag(tau, cartesian)
    pr = _zeros_prims(grid, tau)
    pr.e[:] = e_mean * np.exp(e_amp * field_())
    pr.u[1] = u_amp * field_()
    pr.u[2] = u_amp * field_()
    pr.u[3] = (ueta_amp * field_()) / (1.0 if cartesian else tau)
    pr.u[0] = np.sqrt(1.0 - (g_lo[1] * pr.u[1] ** 2 + g_lo[2] * pr.u[2] ** 2 + g_lo[3] * pr.u[3] ** 2))
    # transverse traceless projection of a random symmetric tensor A^{ab}
    A = np.zeros((4, 4) + grid.shape)
    for a_ in range(4):
        for b_ in range(a_, 4):
            A[a_, b_] = A[b_, a_] = field_() * math.sqrt(abs(g_hi[a_] * g_hi[b_]))
    u = pr.u
    D = np.zeros((4, 4) + grid.shape)   # Delta^mu_nu (mixed)
    for m in range(4):
        for nn in range(4):
            D[m, nn] = (1.0 if m == nn else 0.0) - u[m] * (g_lo[nn] * u[nn])
    # P^{mu nu} = D^mu_a D^nu_b A^{ab}; then remove the trace: - (1/3) Delta^{mu nu} P^a_a
    P = np.einsum("ma...,nb...,ab...->mn...", D, D, A)
    tr = sum(P[a_, a_] * g_lo[a_] for a_ in range(4))
    Dhi = np.zeros((4, 4) + grid.shape)
    for m in range(4):
        for nn in range(4):
            Dhi[m, nn] = (g_hi[m] if m == nn else 0.0) - u[m] * u[nn]
    P = P - Dhi * tr / 3.0
    scale = pi_rel * (4.0 / 3.0) * pr.e
    for m in range(4):
        for nn in range(m, 4):
            pr.pi[pi_component(m, nn)] = scale * P[m, nn]
    pr.Pi[:] = Pi_rel * pr.e * field_()
    pr.meta.update(kind="random_smooth", seed=seed, cartesian=cartesian)
    return pr


# --------------------------------------------------------------------------
# Workload presets: grid, physics configuration, EOS and initial primitives
# --------------------------------------------------------------------------

E_FLOOR_GEV = 1e-7


def default_config(**kw) -> dict:
    """Physics configuration shared by every consumer (plain data)."""
    cfg = dict(dtau=0.01, cartesian=False, periodic=(False, False, False), theta=1.0,
               eta_s=0.0, zeta_coef=0.0, taupipi=10.0 / 7.0, regulate=True, xi0=0.1,
               rho_max=1.0, e_floor=E_FLOOR_GEV / HBARC, newton_tol=1e-12, newton_max=50,
               regulate_bulk=True, m2_delta=1e-3, floor_resets_q=True,
               zeta_model=0, zeta_tc=0.2 / HBARC)
    cfg.update(kw)
    return cfg


@dataclass
class Workload:
    name: str
    grid: Grid
    tau0: float
    n_steps: int
    config: dict
    eos: EOS
    prims: Primitives


def workload_gubser_viscous(n: int = 32, n_steps: int = 50, dx: float = 0.1,
                            deta: float = 0.1, dtau: float = 0.01, eta_s: float = 0.2,
                            theta: float = 1.8, neta: int | None = None) -> Workload:
    """Viscous Gubser flow, conformal 16-d.o.f. EOS, eta/s = 0.2, no bulk,
    tau_pipi = 0, q = 1 fm^-1, tau0 = 1 fm/c, periodic in eta, outflow in x, y."""
    grid = Grid(n, n, n if neta is None else neta, dx, dx, deta)
    cfg = default_config(dtau=dtau, periodic=(False, False, True), theta=theta,
                         eta_s=eta_s, taupipi=0.0, e_floor=1e-8)
    prims = gubser_fields(grid, 1.0, eta_s=eta_s, tau0=1.0)
    return Workload("gubser_viscous_%dx%dx%d" % (grid.nx, grid.ny, grid.neta), grid, 1.0,
                    n_steps, cfg, eos_conformal(), prims)


def workload_hotspot(nx: int = 128, ny: int = 128, neta: int = 128, dx: float = 0.16,
                     deta: float = 0.1, n_steps: int = 200, seed: int = 1, n_hot: int = 200,
                     eos: EOS | None = None) -> Workload:
    """Non-conformal viscous event: shear (eta/s = 0.2) and bulk
    (zeta/s = 0.1 (1/3 - c_s^2)), tabulated EOS, Gaussian hot spots at
    Woods-Saxon positions, tau0 = 0.5 fm/c, dtau = 0.01 fm/c, theta = 1."""
    grid = Grid(nx, ny, neta, dx, dx, deta)
    cfg = default_config(dtau=0.01, theta=1.0, eta_s=0.2, zeta_coef=0.1, taupipi=10.0 / 7.0)
    prims = hotspot_event(grid, tau0=0.5, n_hot=n_hot, seed=seed)
    return Workload("hotspot_viscous_%dx%dx%d" % (nx, ny, neta), grid, 0.5, n_steps, cfg,
                    eos if eos is not None else eos_c1_table(), prims)


# --------------------------------------------------------------------------
# Learned inversion start: seeded initial parameters of the 11-64-64-4 network
# --------------------------------------------------------------------------

MLP_LAYERS = ((64, 11), (64, 64), (4, 64))   # (fan_out, fan_in) of W1, W2, W3
MLP_N_PARAMS = sum(o * i + o for o, i in MLP_LAYERS)   # 5188


def mlp_init_params(seed: int = 0, y0_bias: float = 0.8) -> np.ndarray:
    """Flat float32 vector W1, b1, W2, b2, W3, b3 (row-major weights): weights
    normal with variance 1/fan_in, biases zero except the first output
    (e/E starts near y0_bias)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (fo, fi) in enumerate(MLP_LAYERS):
        parts.append(rng.standard_normal((fo, fi)) / math.sqrt(fi))
        b = np.zeros(fo)
        if k == len(MLP_LAYERS) - 1:
            b[0] = y0_bias
        parts.append(b)
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


# --------------------------------------------------------------------------
# Batches of fluctuating events
# --------------------------------------------------------------------------

BATCH_SHAPES = ((64, 64, 64), (96, 96, 64), (128, 128, 96), (160, 160, 64))


def batch_shapes(n_events: int = 48, seed: int = 7):
    """Grid shape index (into BATCH_SHAPES) and hot-spot count of each event of
    the batch workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = rng.integers(0, len(BATCH_SHAPES), n_events)
    hots = rng.integers(50, 401, n_events)
    return shapes, hots


def workload_batch(n_events: int = 48, seed: int = 7, mixed: bool = True, only=None):
    """Hot-spot events of the 128^3 event's physics on uneven grids: shapes
    drawn uniformly from BATCH_SHAPES (PCG64(seed)), hot-spot counts uniform
    in [50, 400], event k seeded 1000 + k; FP32 state when mixed.  only: the
    indices of the events to build (the same events as in the full set)."""
    shapes, hots = batch_shapes(n_events, seed)
    out = []
    for k in (range(n_events) if only is None else only):
        nx, ny, ne = BATCH_SHAPES[shapes[k]]
        w = workload_hotspot(nx=nx, ny=ny, neta=ne, n_hot=int(hots[k]), seed=1000 + k)
        if mixed:
            w.config["mixed"] = True
        out.append(w)
    return out
