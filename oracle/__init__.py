"""ctypes binding of the plain FP64 CPU oracle (``kt_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  It never imports the HIP library and
the HIP library never imports it.

Arrays are arrays of structures: ``q`` is (ncell, 15) with the component
order of Sec. 3.1 (T^{tau mu}, pi^{tt,tx,ty,te,xx,xy,xe,yy,ye,ee}, Pi), ``u``
is (ncell, 4); the cell index runs x fastest, eta slowest.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NQ = 15


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP over cells)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                        "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("neta", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("deta", C.c_double),
                ("dtau", C.c_double), ("cartesian", C.c_int32), ("periodic", C.c_int32 * 3),
                ("theta", C.c_double), ("eta_s", C.c_double), ("zeta_coef", C.c_double),
                ("taupipi", C.c_double), ("regulate", C.c_int32), ("xi0", C.c_double),
                ("rho_max", C.c_double), ("e_floor", C.c_double), ("newton_tol", C.c_double),
                ("newton_max", C.c_int32), ("regulate_bulk", C.c_int32),
                ("m2_delta", C.c_double), ("floor_resets_q", C.c_int32),
                ("zeta_model", C.c_int32), ("zeta_tc", C.c_double)]


class _EOS(C.Structure):
    _fields_ = [("conformal", C.c_int32), ("a_sb", C.c_double), ("n", C.c_int32),
                ("ln_e0", C.c_double), ("dln", C.c_double),
                ("p", C.POINTER(C.c_double)), ("cs2", C.POINTER(C.c_double)),
                ("T", C.POINTER(C.c_double))]


class _Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int64), ("n_recover", C.c_int64), ("n_floor", C.c_int64),
                ("n_clamp", C.c_int64), ("n_fallback", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        P, E = C.POINTER(_Params), C.POINTER(_EOS)
        L.ora_tmunu.argtypes = [P, E, C.c_double, C.c_int64, dp, dp, dp, dp, dp]
        L.ora_recover.argtypes = [P, E, C.c_double, C.c_int64, dp, C.c_void_p, dp, dp, ip, ip]
        L.ora_regulate.argtypes = [P, E, C.c_double, C.c_int64, dp, dp, dp, dp]
        L.ora_eos_eval.argtypes = [E, C.c_int64, dp, dp, dp, dp]
        L.ora_zeta_over_s_paper.argtypes = [C.c_double]
        L.ora_zeta_over_s_paper.restype = C.c_double
        L.ora_init.argtypes = [P, E, C.c_double, dp, dp, dp, dp]
        L.ora_rhs.argtypes = [P, E, C.c_double, dp, dp, dp, dp, dp]
        L.ora_step.argtypes = [P, E, dp, dp, dp, dp, dp, C.c_int32, C.POINTER(_Stats)]
        L.ora_step.restype = C.c_int
        L.ora_kinematics.argtypes = [C.c_double, C.c_int32, dp, dp, dp]
        L.ora_second_order.argtypes = [C.c_double, C.c_int32, dp, dp, dp, dp]
        L.ora_gpi.argtypes = [C.c_double, C.c_int32, dp, dp, dp]
        L.ora_minmod3.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_minmod3.restype = C.c_double
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int32]
        L.ora_observables.argtypes = [P, E, C.c_double, dp, dp, dp, dp]
        L.ora_validity2.argtypes = [P, E, C.c_double, dp, dp, dp, dp, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        L.ora_expand.argtypes = [P, C.c_double, C.c_int64, dp, dp, dp, dp]
        L.ora_pi_dependent.argtypes = [C.c_double, C.c_int32, C.c_int64, dp, dp]
        L.ora_recover_reduced.argtypes = [P, E, C.c_double, C.c_int64, dp, dp, dp, ip, ip, ip]
        L.ora_init_reduced.argtypes = [P, E, C.c_double, dp, dp, dp, dp]
        L.ora_step_reduced.argtypes = [P, E, dp, dp, dp, dp, dp, dp, C.c_int32, C.POINTER(_Stats),
                                       C.POINTER(C.c_int64)]
        L.ora_step_reduced.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


@dataclass
class Physics:
    """Grid and physics parameters of one run (the oracle's own copy)."""
    nx: int
    ny: int
    neta: int
    dx: float
    dy: float
    deta: float
    dtau: float
    cartesian: bool = False
    periodic: tuple = (False, False, False)
    theta: float = 1.0
    eta_s: float = 0.0
    zeta_coef: float = 0.0
    taupipi: float = 10.0 / 7.0
    regulate: bool = True
    xi0: float = 0.1
    rho_max: float = 1.0
    e_floor: float = 1e-7 / 0.1973269804
    newton_tol: float = 1e-12
    newton_max: int = 50
    regulate_bulk: bool = True
    m2_delta: float = 1e-3
    floor_resets_q: bool = True
    zeta_model: int = 0
    zeta_tc: float = 0.2 / 0.1973269804

    @classmethod
    def from_config(cls, grid, cfg: dict):
        keys = cls.__dataclass_fields__.keys()
        kw = {k: v for k, v in cfg.items() if k in keys}
        return cls(nx=grid.nx, ny=grid.ny, neta=grid.neta, dx=grid.dx, dy=grid.dy,
                   deta=grid.deta, **kw)

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.neta, self.dx, self.dy, self.deta, self.dtau,
                       int(self.cartesian), (C.c_int32 * 3)(*[int(b) for b in self.periodic]),
                       self.theta, self.eta_s, self.zeta_coef, self.taupipi, int(self.regulate),
                       self.xi0, self.rho_max, self.e_floor, self.newton_tol, self.newton_max,
                       int(self.regulate_bulk), self.m2_delta, int(self.floor_resets_q),
                       int(self.zeta_model), self.zeta_tc)

    @property
    def ncells(self):
        return self.nx * self.ny * self.neta


class EOSRef:
    """Holds the C view of an EOS description (keeps the arrays alive)."""

    def __init__(self, eos):
        self.eos = eos
        if eos.conformal:
            self._arrs = ()
            self.c = _EOS(1, eos.a_sb, 0, 0.0, 0.0, None, None, None)
        else:
            self._arrs = tuple(np.ascontiguousarray(a, dtype=np.float64) for a in (eos.p, eos.cs2, eos.T))
            self.c = _EOS(0, eos.a_sb, len(self._arrs[0]), eos.ln_e0, eos.dln_e,
                          *[_dp(a) for a in self._arrs])


def eos_eval(eos, e):
    ref = EOSRef(eos)
    e = np.ascontiguousarray(e, dtype=np.float64).ravel()
    p, c2, T = np.empty_like(e), np.empty_like(e), np.empty_like(e)
    lib().ora_eos_eval(C.byref(ref.c), e.size, _dp(e), _dp(p), _dp(c2), _dp(T))
    return p, c2, T


def validity_maps(eos, tau, cartesian, e, pi, Pi):
    """Sec. 7 (Eq. inverseReynoldsNumbers): T(e), sqrt(pi^{mu nu} pi_{mu nu})/P(e)
    and |Pi|/P(e) per cell.  pi: the ten contravariant components in the order
    tt, tx, ty, te, xx, xy, xe, yy, ye, ee (leading axis); both indices are
    lowered with diag(1, -1, -1, -tau^2) (Milne) or diag(1, -1, -1, -1)."""
    e = np.asarray(e, dtype=np.float64)
    p, _, T = eos_eval(eos, e)
    p, T = p.reshape(e.shape), T.reshape(e.shape)
    g = np.array([1.0, -1.0, -1.0, -1.0 if cartesian else -tau * tau])
    full = np.zeros((4, 4) + e.shape)
    pairs = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    for k, (m, n) in enumerate(pairs):
        full[m, n] = pi[k]
        full[n, m] = pi[k]
    pp = np.einsum("m,n,mn...,mn...->...", g, g, full, full)
    return T, np.sqrt(np.maximum(pp, 0.0)) / p, np.abs(np.asarray(Pi)) / p


OBS_KEYS = ("energy", "momentum_x", "momentum_y", "momentum_eta", "e_max", "T_max", "v_max",
            "cfl", "norm_err", "pi_transverse", "pi_trace", "n_nan")


def observables(phys: "Physics", eos, tau, q, e, u) -> dict:
    """The state's observables (the definitions of the library's kt_obs): sums
    of T^{tau mu} times the cell volume, maxima of e, T, |v|, the CFL number,
    |u.u - 1| and the pi-constraint ratios of Sec. 2.4, non-finite cells."""
    ref = EOSRef(eos)
    out = np.empty(12)
    P = phys.c()
    lib().ora_observables(C.byref(P), C.byref(ref.c), float(tau), _dp(np.ascontiguousarray(q, float)),
                          _dp(np.ascontiguousarray(e, float)), _dp(np.ascontiguousarray(u, float)),
                          _dp(out))
    return dict(zip(OBS_KEYS, out))


def validity2(phys: "Physics", eos, tau, q, e, u, up):
    """Per cell (AoS state as in Simulation): the second-order inverse Reynolds
    numbers of Sec. 7 (Eq. inverseReynoldsNumbers2) and the regulation factor
    tanh(rho)/rho of Sec. 3.2 evaluated on the state."""
    ref = EOSRef(eos)
    n = phys.ncells
    r2pi, r2Pi, reg = np.empty(n), np.empty(n), np.empty(n)
    P = phys.c()
    lib().ora_validity2(C.byref(P), C.byref(ref.c), float(tau), _dp(np.ascontiguousarray(q, float)),
                        _dp(np.ascontiguousarray(e, float)), _dp(np.ascontiguousarray(u, float)),
                        _dp(np.ascontiguousarray(up, float)), r2pi.ctypes.data_as(C.c_void_p),
                        r2Pi.ctypes.data_as(C.c_void_p), reg.ctypes.data_as(C.c_void_p))
    return r2pi, r2Pi, reg


def zeta_over_s_paper(x):
    """The oracle's zeta/s(T / T_c) of Sec. 2.2 (Eq. zetas), elementwise."""
    return np.array([lib().ora_zeta_over_s_paper(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def aos_from_prims(prims):
    """(ncell,) e, (ncell,4) u, (ncell,10) pi, (ncell,) Pi from component-first arrays."""
    n = prims.e.size
    e = np.ascontiguousarray(prims.e.reshape(n), dtype=np.float64)
    u = np.ascontiguousarray(prims.u.reshape(4, n).T, dtype=np.float64)
    pi = np.ascontiguousarray(prims.pi.reshape(10, n).T, dtype=np.float64)
    Pi = np.ascontiguousarray(prims.Pi.reshape(n), dtype=np.float64)
    return e, u, pi, Pi


def tmunu(phys: Physics, eos, tau, e, u, pi, Pi):
    ref = EOSRef(eos)
    n = e.shape[0]
    q = np.empty((n, NQ))
    P = phys.c()
    lib().ora_tmunu(C.byref(P), C.byref(ref.c), tau, n, _dp(e), _dp(u), _dp(pi), _dp(Pi), _dp(q))
    return q


def recover(phys: Physics, eos, tau, q, e_start=None):
    """Cell inversion of q (n, 15) at tau; e_start (n,) optional Newton start
    (values <= 0: the conformal closed form, the default)."""
    ref = EOSRef(eos)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0]
    e = np.empty(n)
    u = np.empty((n, 4))
    it = np.empty(n, np.int32)
    fl = np.empty(n, np.int32)
    P = phys.c()
    es = None
    if e_start is not None:
        es = np.ascontiguousarray(e_start, dtype=np.float64)
        assert es.shape == (n,)
    lib().ora_recover(C.byref(P), C.byref(ref.c), tau, n, _dp(q),
                      None if es is None else es.ctypes.data_as(C.c_void_p),
                      _dp(e), _dp(u), _ip(it), _ip(fl))
    return e, u, it, fl


def regulate(phys: Physics, eos, tau, q, e, u):
    ref = EOSRef(eos)
    q = np.array(q, dtype=np.float64, order="C")
    fac = np.empty(q.shape[0])
    P = phys.c()
    lib().ora_regulate(C.byref(P), C.byref(ref.c), tau, q.shape[0], _dp(q),
                       _dp(np.ascontiguousarray(e)), _dp(np.ascontiguousarray(u)), _dp(fac))
    return q, fac


def kinematics(tau, cartesian, u, du):
    out = np.empty(53)
    lib().ora_kinematics(tau, int(cartesian), _dp(np.ascontiguousarray(u, float)),
                         _dp(np.ascontiguousarray(du, float).ravel()), _dp(out))
    return dict(theta=out[0], sigma=out[1:17].reshape(4, 4), omega=out[17:33].reshape(4, 4),
                Du_lo=out[33:37], Delta=out[37:53].reshape(4, 4))


def second_order(tau, cartesian, u, du, pi16):
    out = np.empty(65)
    lib().ora_second_order(tau, int(cartesian), _dp(np.ascontiguousarray(u, float)),
                           _dp(np.ascontiguousarray(du, float).ravel()),
                           _dp(np.ascontiguousarray(pi16, float).ravel()), _dp(out))
    return dict(I1=out[0:16].reshape(4, 4), I2=out[16:32].reshape(4, 4),
                I3=out[32:48].reshape(4, 4), I4=out[48:64].reshape(4, 4), pi_sigma=out[64])


def gpi(tau, cartesian, u, pi16):
    out = np.empty(16)
    lib().ora_gpi(tau, int(cartesian), _dp(np.ascontiguousarray(u, float)),
                  _dp(np.ascontiguousarray(pi16, float).ravel()), _dp(out))
    return out.reshape(4, 4)


def minmod3(x, y, z):
    return lib().ora_minmod3(float(x), float(y), float(z))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (results do not depend on it)."""
    lib().ora_set_num_threads(int(n))


class Simulation:
    """Oracle state: q, e, u, u_prev (AoS) and tau; steps in place."""

    def __init__(self, phys: Physics, eos, tau0: float, q: np.ndarray):
        self.phys = phys
        self.eos_ref = EOSRef(eos)
        self.tau = float(tau0)
        n = phys.ncells
        self.q = np.array(q, dtype=np.float64, order="C").reshape(n, NQ)
        self.e = np.empty(n)
        self.u = np.empty((n, 4))
        self.up = np.empty((n, 4))
        self.step_count = 0
        self.stats = _Stats()
        self._P = phys.c()
        lib().ora_init(C.byref(self._P), C.byref(self.eos_ref.c), self.tau, _dp(self.q),
                       _dp(self.e), _dp(self.u), _dp(self.up))

    @classmethod
    def from_primitives(cls, phys: Physics, eos, prims):
        e, u, pi, Pi = aos_from_prims(prims)
        q = tmunu(phys, eos, prims.tau0, e, u, pi, Pi)
        return cls(phys, eos, prims.tau0, q)

    def step(self, n: int = 1):
        tau = C.c_double(self.tau)
        rc = lib().ora_step(C.byref(self._P), C.byref(self.eos_ref.c), C.byref(tau), _dp(self.q),
                            _dp(self.e), _dp(self.u), _dp(self.up), int(n), C.byref(self.stats))
        if rc != 0:
            raise MemoryError("oracle step could not allocate its work arrays")
        self.tau = tau.value
        self.step_count += n
        return self

    def rhs(self):
        out = np.empty_like(self.q)
        lib().ora_rhs(C.byref(self._P), C.byref(self.eos_ref.c), self.tau, _dp(self.q),
                      _dp(self.e), _dp(self.u), _dp(self.up), _dp(out))
        return out

    # component-first views for comparisons
    def shape(self):
        return (self.phys.neta, self.phys.ny, self.phys.nx)

    def fields(self):
        s = self.shape()
        return dict(e=self.e.reshape(s).copy(),
                    u=self.u.T.reshape((4,) + s).copy(),
                    up=self.up.T.reshape((4,) + s).copy(),
                    q=self.q.T.reshape((NQ,) + s).copy())


# ------------------------------------------------------------ reduced storage --
#: positions in the 15-component q of the reduced evolved vector
#: (T^{tau mu}, pi^{xx}, pi^{xy}, pi^{x eta}, pi^{yy}, pi^{y eta}, Pi)
RED_IDX = (0, 1, 2, 3, 8, 9, 10, 11, 12, 14)
NR = len(RED_IDX)


def pi_dependent(tau, cartesian, u, q):
    """q (n, 15) with pi^{tau mu} and pi^{eta eta} replaced by the values that
    Eqs. pi_tautau .. pi_etaeta (Sec. 2.4) give from the five independent
    components and u (n, 4)."""
    q = np.array(q, dtype=np.float64, order="C")
    u = np.ascontiguousarray(u, dtype=np.float64)
    lib().ora_pi_dependent(float(tau), int(cartesian), q.shape[0], _dp(u), _dp(q))
    return q


def recover_reduced(phys: Physics, eos, tau, r):
    """Recovery of n reduced states r (n, 10): e, u (n, 4), Newton iterations,
    fixed-point passes (negative where the fixed point did not converge), flags."""
    ref = EOSRef(eos)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    e, u = np.empty(n), np.empty((n, 4))
    it, ps, fl = (np.empty(n, np.int32) for _ in range(3))
    P = phys.c()
    lib().ora_recover_reduced(C.byref(P), C.byref(ref.c), float(tau), n, _dp(r), _dp(e), _dp(u),
                              _ip(it), _ip(ps), _ip(fl))
    return e, u, it, ps, fl


class ReducedSimulation:
    """Oracle state with reduced storage (Sec. 2.4: five pi components and three
    u components; the rest rebuilt algebraically): r (n, 10), e, u3 (n, 3),
    up3 and tau; steps in place.  fields() expands to all components."""

    def __init__(self, phys: Physics, eos, tau0: float, q: np.ndarray):
        self.phys = phys
        self.eos_ref = EOSRef(eos)
        self.tau = float(tau0)
        n = phys.ncells
        q = np.asarray(q, dtype=np.float64).reshape(n, NQ)
        self.r = np.ascontiguousarray(q[:, list(RED_IDX)])
        self.e = np.empty(n)
        self.u3 = np.empty((n, 3))
        self.up3 = np.empty((n, 3))
        self.step_count = 0
        self.tau_prev = float(tau0)           # time of u_prev's level (u^{-1} = u^0 before the first step)
        self.stats = _Stats()
        self.fp = np.zeros(2, np.int64)       # fixed-point passes, cells not converged
        self._P = phys.c()
        lib().ora_init_reduced(C.byref(self._P), C.byref(self.eos_ref.c), self.tau, _dp(self.r),
                               _dp(self.e), _dp(self.u3), _dp(self.up3))

    @classmethod
    def from_primitives(cls, phys: Physics, eos, prims):
        e, u, pi, Pi = aos_from_prims(prims)
        q = tmunu(phys, eos, prims.tau0, e, u, pi, Pi)
        return cls(phys, eos, prims.tau0, q)

    def step(self, n: int = 1):
        tau, tau_prev = C.c_double(self.tau), C.c_double(self.tau_prev)
        rc = lib().ora_step_reduced(C.byref(self._P), C.byref(self.eos_ref.c), C.byref(tau),
                                    C.byref(tau_prev), _dp(self.r), _dp(self.e), _dp(self.u3), _dp(self.up3), int(n),
                                    C.byref(self.stats), self.fp.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != 0:
            raise MemoryError("oracle step could not allocate its work arrays")
        self.tau = tau.value
        self.tau_prev = tau_prev.value
        self.step_count += n
        return self

    def expanded(self, tau=None, u3=None):
        """Full q (n, 15) and u (n, 4) of the state (u3 at tau, default the current)."""
        n = self.phys.ncells
        q, u = np.empty((n, NQ)), np.empty((n, 4))
        u3 = self.u3 if u3 is None else np.ascontiguousarray(u3)
        lib().ora_expand(C.byref(self._P), float(self.tau if tau is None else tau), n, _dp(self.r),
                         _dp(u3), _dp(q), _dp(u))
        return q, u

    def shape(self):
        return (self.phys.neta, self.phys.ny, self.phys.nx)

    def fields(self):
        s = self.shape()
        q, u = self.expanded()
        _, up = self.expanded(self.tau_prev, self.up3)
        return dict(e=self.e.reshape(s).copy(), u=u.T.reshape((4,) + s).copy(),
                    up=up.T.reshape((4,) + s).copy(), q=q.T.reshape((NQ,) + s).copy())
