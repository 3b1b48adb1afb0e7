"""ctypes binding of ``libkt.so`` (the C ABI declared in ``include/kt.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies device memory (the workspace and the field
tensors) and the stream.  Importing this module does not load the library;
the first use does, and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkt.so")

KT_OK, KT_E_ARG, KT_E_ALLOC, KT_E_HIP, KT_E_STATE, KT_E_UNSUPPORTED = range(6)
KT_FP64, KT_MIXED = 0, 1
KT_MILNE, KT_CARTESIAN = 0, 1
KT_BC_OUTFLOW, KT_BC_PERIODIC = 0, 1
NQ = 15

_dp = C.POINTER(C.c_double)


class KtEos(C.Structure):
    _fields_ = [("conformal", C.c_int32), ("a_sb", C.c_double), ("n", C.c_int32),
                ("ln_e0", C.c_double), ("dln_e", C.c_double),
                ("p", _dp), ("cs2", _dp), ("T", _dp)]


class KtParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("neta", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("deta", C.c_double),
                ("tau0", C.c_double), ("dtau", C.c_double), ("coords", C.c_int32),
                ("bc", C.c_int32 * 3), ("theta", C.c_double), ("eta_over_s", C.c_double),
                ("zeta_coef", C.c_double), ("taupipi", C.c_double), ("regulate", C.c_int32),
                ("regulate_bulk", C.c_int32), ("xi0", C.c_double), ("rho_max", C.c_double),
                ("e_floor", C.c_double), ("m2_delta", C.c_double), ("floor_resets_q", C.c_int32),
                ("newton_tol", C.c_double), ("newton_max", C.c_int32), ("precision", C.c_int32),
                ("zeta_model", C.c_int32), ("zeta_tc", C.c_double), ("reduced", C.c_int32)]


class KtInitState(C.Structure):
    _fields_ = [("q", C.c_void_p * 15), ("e", C.c_void_p), ("u", C.c_void_p * 4),
                ("pi", C.c_void_p * 10), ("Pi", C.c_void_p), ("u_prev", C.c_void_p * 4),
                ("p", C.c_void_p)]


class KtFields(C.Structure):
    _fields_ = [("e", C.c_void_p), ("u", C.c_void_p * 4), ("q", C.c_void_p * 15),
                ("u_prev", C.c_void_p * 4), ("p", C.c_void_p)]


class KtObs(C.Structure):
    _fields_ = [("tau", C.c_double), ("step", C.c_int64), ("energy", C.c_double),
                ("momentum", C.c_double * 3), ("e_max", C.c_double), ("T_max", C.c_double),
                ("v_max", C.c_double), ("cfl", C.c_double), ("norm_err", C.c_double),
                ("pi_transverse", C.c_double), ("pi_trace", C.c_double), ("n_nan", C.c_int64),
                ("newton_iters_cells", C.c_int64), ("n_recover_cells", C.c_int64),
                ("newton_iters_faces", C.c_int64), ("n_recover_faces", C.c_int64),
                ("n_floor", C.c_int64), ("n_clamp", C.c_int64), ("n_fallback", C.c_int64),
                ("n_fallback_faces", C.c_int64), ("fp_passes", C.c_int64),
                ("fp_not_converged", C.c_int64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "momentum" else v
        return d


class KtProfile(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_int64 * 4)]


class KtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("kt status %d: %s" % (status, msg))
        self.status = status


_lib = None

#: every function the C ABI exports (the names declared in include/kt.h)
EXPORTS = ("kt_workspace_bytes", "kt_init", "kt_init_static", "kt_step", "kt_recover", "kt_recover_reduced",
           "kt_observables",
           "kt_validity", "kt_run_to_freezeout",
           "kt_profile_enable", "kt_profile_read", "kt_destroy", "kt_last_error",
           "kt_status_string", "kt_set_inv_start", "kt_mlp_set", "kt_mlp_get", "kt_mlp_features",
           "kt_mlp_fwd", "kt_mlp_y0", "kt_mlp_loss", "kt_mlp_bwd", "kt_mlp_adam", "kt_batch_workspace_bytes",
           "kt_batch_init", "kt_batch_step", "kt_batch_tune", "kt_batch_set_flux_blocks",
           "kt_batch_observables",
           "kt_batch_destroy", "kt_batch_last_error")

KT_START_WARM, KT_START_CONFORMAL, KT_START_LEARNED = 0, 1, 2
KT_MLP_NPARAMS = 5188


# kernel classes of kt_profile (include/kt.h)
PROFILE_CLASSES = ("flux", "recover", "faces", "sources")


def lib():
    """Load libkt.so; raises if the library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkt.so is missing: run __graft_entry__.build() first (%s)" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        L.kt_workspace_bytes.argtypes = [C.POINTER(KtParams), C.POINTER(KtEos)]
        L.kt_workspace_bytes.restype = C.c_size_t
        L.kt_init.argtypes = [C.POINTER(KtParams), C.POINTER(KtEos), C.POINTER(KtInitState),
                              C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.kt_init_static.argtypes = [C.POINTER(KtParams), C.POINTER(KtEos), C.POINTER(KtInitState),
                                     C.c_void_p, C.POINTER(C.c_void_p)]
        L.kt_step.argtypes = [C.c_void_p, C.c_int32]
        L.kt_recover.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p * 9, C.c_void_p,
                                 C.c_void_p * 4, C.c_void_p, C.c_void_p]
        L.kt_recover_reduced.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p * 10, C.c_void_p,
                                         C.c_void_p * 4, C.POINTER(C.c_void_p * 5), C.c_void_p, C.c_void_p]
        L.kt_observables.argtypes = [C.c_void_p, C.POINTER(KtObs), C.POINTER(KtFields)]
        L.kt_validity.argtypes = [C.c_void_p] + [C.c_void_p] * 8
        L.kt_run_to_freezeout.argtypes = [C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_int32)]
        L.kt_destroy.argtypes = [C.c_void_p]
        L.kt_destroy.restype = None
        L.kt_last_error.argtypes = [C.c_void_p]
        L.kt_last_error.restype = C.c_char_p
        L.kt_status_string.argtypes = [C.c_int]
        L.kt_status_string.restype = C.c_char_p
        L.kt_profile_enable.argtypes = [C.c_void_p, C.c_int32]
        L.kt_profile_read.argtypes = [C.c_void_p, C.POINTER(KtProfile)]
        vp = C.c_void_p
        L.kt_set_inv_start.argtypes = [vp, C.c_int32]
        L.kt_mlp_set.argtypes = [vp, vp, C.c_int32]
        L.kt_mlp_get.argtypes = [vp, vp, C.c_int32]
        L.kt_mlp_features.argtypes = [vp, C.c_int64, C.c_double, vp * 9, vp, vp, vp, vp]
        L.kt_mlp_fwd.argtypes = [vp, C.c_int64, vp, vp, vp]
        L.kt_mlp_y0.argtypes = [vp, C.c_int64, vp, vp]
        L.kt_mlp_loss.argtypes = [vp, C.c_int64, vp, vp, C.POINTER(C.c_float), vp, vp]
        L.kt_mlp_bwd.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.kt_mlp_adam.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]
        L.kt_batch_workspace_bytes.argtypes = [C.POINTER(KtParams), C.c_int32, C.POINTER(KtEos)]
        L.kt_batch_workspace_bytes.restype = C.c_size_t
        L.kt_batch_init.argtypes = [C.POINTER(KtParams), C.c_int32, C.POINTER(KtEos),
                                    C.POINTER(KtInitState), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.kt_batch_step.argtypes = [vp, C.c_int32]
        L.kt_batch_tune.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.kt_batch_set_flux_blocks.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.kt_batch_observables.argtypes = [vp, C.c_int32, C.POINTER(KtObs), C.POINTER(KtFields)]
        L.kt_batch_destroy.argtypes = [vp]
        L.kt_batch_destroy.restype = None
        L.kt_batch_last_error.argtypes = [vp]
        L.kt_batch_last_error.restype = C.c_char_p
        for f in ("kt_batch_init", "kt_batch_step", "kt_batch_tune", "kt_batch_set_flux_blocks",
                  "kt_batch_observables"):
            getattr(L, f).restype = C.c_int
        for f in ("kt_validity", "kt_run_to_freezeout"):
            getattr(L, f).restype = C.c_int
        for f in ("kt_init", "kt_init_static", "kt_step", "kt_recover", "kt_recover_reduced", "kt_observables", "kt_profile_enable",
                  "kt_profile_read", "kt_set_inv_start", "kt_mlp_set", "kt_mlp_get",
                  "kt_mlp_features", "kt_mlp_fwd", "kt_mlp_y0", "kt_mlp_loss", "kt_mlp_bwd", "kt_mlp_adam"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != KT_OK:
        msg = lib().kt_last_error(ctx).decode(errors="replace")
        raise KtError(status, msg)


def make_params(grid, config: dict, tau0: float) -> KtParams:
    per = config.get("periodic", (False, False, False))
    return KtParams(
        grid.nx, grid.ny, grid.neta, grid.dx, grid.dy, grid.deta, tau0, config["dtau"],
        KT_CARTESIAN if config.get("cartesian", False) else KT_MILNE,
        (C.c_int32 * 3)(*[KT_BC_PERIODIC if b else KT_BC_OUTFLOW for b in per]),
        config.get("theta", 1.0), config.get("eta_s", 0.0), config.get("zeta_coef", 0.0),
        config.get("taupipi", 10.0 / 7.0), int(config.get("regulate", True)),
        int(config.get("regulate_bulk", True)), config.get("xi0", 0.1),
        config.get("rho_max", 1.0), config["e_floor"], config.get("m2_delta", 1e-3),
        int(config.get("floor_resets_q", True)), config.get("newton_tol", 1e-12),
        int(config.get("newton_max", 50)), KT_MIXED if config.get("mixed", False) else KT_FP64,
        int(config.get("zeta_model", 0)), config.get("zeta_tc", 0.2 / 0.1973269804),
        int(config.get("reduced", False)))


class EosHost:
    """Host-side C view of an EOS description (keeps the arrays alive)."""

    def __init__(self, eos):
        if eos.conformal:
            self._arrs = ()
            self.c = KtEos(1, eos.a_sb, 0, 0.0, 0.0, None, None, None)
        else:
            self._arrs = tuple(np.ascontiguousarray(a, dtype=np.float64) for a in (eos.p, eos.cs2, eos.T))
            self.c = KtEos(0, eos.a_sb, len(self._arrs[0]), eos.ln_e0, eos.dln_e,
                           *[a.ctypes.data_as(_dp) for a in self._arrs])


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def workspace_bytes(grid, config, eos, tau0=1.0) -> int:
    p = make_params(grid, config, tau0)
    e = EosHost(eos)
    return int(lib().kt_workspace_bytes(C.byref(p), C.byref(e.c)))


def _init_state(torch, device, grid, prims, q, u_prev, keep, resume=None) -> KtInitState:
    """Device arrays of an initial state (kept alive in keep) as a KtInitState.
    resume: dict with e, u and optionally p (with q: the state taken as given)."""
    st = KtInitState()
    shape = grid.shape

    def dev(a):
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device) \
            if isinstance(a, np.ndarray) else a.contiguous()
        assert t.dtype == torch.float64 and tuple(t.shape[-3:]) == shape
        keep.append(t)
        return t

    if q is not None:
        qd = dev(q)
        for c in range(NQ):
            st.q[c] = qd[c].data_ptr()
    else:
        get = (lambda k: prims[k]) if isinstance(prims, dict) else (lambda k: getattr(prims, k))
        e, u, pi, Pi = dev(get("e")), dev(get("u")), dev(get("pi")), dev(get("Pi"))
        st.e = e.data_ptr()
        st.Pi = Pi.data_ptr()
        for m in range(4):
            st.u[m] = u[m].data_ptr()
        for c in range(10):
            st.pi[c] = pi[c].data_ptr()
    if resume is not None:
        assert q is not None, "resuming needs q"
        ed, ud = dev(resume["e"]), dev(resume["u"])
        st.e = ed.data_ptr()
        for m in range(4):
            st.u[m] = ud[m].data_ptr()
        if resume.get("p") is not None:
            st.p = dev(resume["p"]).data_ptr()
    if u_prev is not None:
        upd = dev(u_prev)
        for m in range(4):
            st.u_prev[m] = upd[m].data_ptr()
    return st


class Solver:
    """One event advanced by the HIP library.

    prims: ``inputs.Primitives`` (numpy, component-first) or a dict of device
    tensors ``e, u, pi, Pi``; alternatively ``q`` = (15, neta, ny, nx) device
    tensor of conserved components, recovered, or with ``resume`` = dict(e, u,
    p) of an exported state (``fields(("e", "p", "u", "q", "u_prev"))``) taken
    as it is, so that the run continues bit for bit at ``tau0``.
    """

    def __init__(self, grid, config: dict, eos, prims=None, q=None, tau0=None, u_prev=None,
                 device="cuda:0", static_workspace=False, resume=None, workspace=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.grid = grid
        self.config = dict(config)
        if tau0 is None:
            tau0 = prims.tau0 if prims is not None and hasattr(prims, "tau0") else 1.0
        self.params = make_params(grid, config, tau0)
        self.eos_host = EosHost(eos)
        L = lib()
        nbytes = int(L.kt_workspace_bytes(C.byref(self.params), C.byref(self.eos_host.c)))
        if nbytes == 0:
            _check(KT_E_ARG)
        with torch.cuda.device(self.device):
            keep = []
            st = _init_state(torch, self.device, grid, prims, q, u_prev, keep, resume)
            stream = torch.cuda.current_stream(self.device).cuda_stream
            ctx = C.c_void_p()
            if static_workspace:
                # the library's static per-GPU workspace (kt_init_static)
                self.ws = None
                _check(L.kt_init_static(C.byref(self.params), C.byref(self.eos_host.c), C.byref(st),
                                        C.c_void_p(stream), C.byref(ctx)))
            else:
                # workspace: a caller's uint8 device tensor of at least kt_workspace_bytes
                # (its contents are not assumed), else a new one
                if workspace is not None:
                    assert workspace.dtype == torch.uint8 and workspace.numel() >= nbytes
                    self.ws = workspace
                else:
                    self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                if self.ws.data_ptr() % 256:
                    raise RuntimeError("workspace is not 256-byte aligned")
                _check(L.kt_init(C.byref(self.params), C.byref(self.eos_host.c), C.byref(st),
                                 C.c_void_p(self.ws.data_ptr()), nbytes, C.c_void_p(stream),
                                 C.byref(ctx)))
            self.ctx = ctx
            del keep

    # ------------------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().kt_step(self.ctx, int(n)), self.ctx)
        return self

    def observables(self) -> dict:
        o = KtObs()
        _check(lib().kt_observables(self.ctx, C.byref(o), None), self.ctx)
        return o.as_dict()

    def validity(self) -> dict:
        """T, R^{-1}_pi, R^{-1}_Pi, Kn_pi, Kn_Pi, the second-order (R^{(2)}_pi)^{-1},
        (R^{(2)}_Pi)^{-1} (Sec. 7) and the regulation factor tanh(rho)/rho (Sec. 3.2)
        per cell, as (neta, ny, nx) tensors."""
        torch = self.torch
        names = ("T", "rinv_pi", "rinv_Pi", "kn_pi", "kn_Pi", "rinv2_pi", "rinv2_Pi", "reg")
        with torch.cuda.device(self.device):
            out = {k: torch.empty(self.grid.shape, dtype=torch.float64, device=self.device) for k in names}
            _check(lib().kt_validity(self.ctx, *[out[k].data_ptr() for k in names]), self.ctx)
            torch.cuda.synchronize(self.device)
        return out

    def run_to_freezeout(self, T_f: float, max_steps: int, check_every: int = 10) -> int:
        """Steps until max T < T_f (checked every check_every steps); returns the steps taken."""
        n = C.c_int32(0)
        _check(lib().kt_run_to_freezeout(self.ctx, float(T_f), int(max_steps), int(check_every),
                                         C.byref(n)), self.ctx)
        return n.value

    def fields(self, which=("e", "u", "q", "u_prev")) -> dict:
        torch = self.torch
        shape = self.grid.shape
        out = {}
        f = KtFields()
        with torch.cuda.device(self.device):
            if "e" in which:
                out["e"] = torch.empty(shape, dtype=torch.float64, device=self.device)
                f.e = out["e"].data_ptr()
            if "p" in which:
                out["p"] = torch.empty(shape, dtype=torch.float64, device=self.device)
                f.p = out["p"].data_ptr()
            if "u" in which:
                out["u"] = torch.empty((4,) + shape, dtype=torch.float64, device=self.device)
                for m in range(4):
                    f.u[m] = out["u"][m].data_ptr()
            if "u_prev" in which:
                out["u_prev"] = torch.empty((4,) + shape, dtype=torch.float64, device=self.device)
                for m in range(4):
                    f.u_prev[m] = out["u_prev"][m].data_ptr()
            if "q" in which:
                out["q"] = torch.empty((NQ,) + shape, dtype=torch.float64, device=self.device)
                for c in range(NQ):
                    f.q[c] = out["q"][c].data_ptr()
            _check(lib().kt_observables(self.ctx, None, C.byref(f)), self.ctx)
        return out

    def recover(self, ins, tau: float, with_iters=True):
        """ins: 9 device tensors (T^{tau mu}, pi^{tau mu}, Pi) of equal length n."""
        torch = self.torch
        n = ins[0].numel()
        arr = (C.c_void_p * 9)(*[t.data_ptr() if t is not None else None for t in ins])
        e = torch.empty(n, dtype=torch.float64, device=self.device)
        u = torch.empty((4, n), dtype=torch.float64, device=self.device)
        it = torch.empty(n, dtype=torch.int32, device=self.device) if with_iters else None
        fl = torch.empty(n, dtype=torch.int32, device=self.device) if with_iters else None
        uarr = (C.c_void_p * 4)(*[u[m].data_ptr() for m in range(4)])
        _check(lib().kt_recover(self.ctx, n, float(tau), arr, C.c_void_p(e.data_ptr()), uarr,
                                _ptr(it), _ptr(fl)), self.ctx)
        return e, u, it, fl

    def recover_reduced(self, ins, tau: float, with_pi=True):
        """ins: 10 device tensors (T^{tau mu}, pi^{xx}, pi^{xy}, pi^{x eta},
        pi^{yy}, pi^{y eta}, Pi or None) of equal length n.  Returns e, u (4, n),
        the five rebuilt components (5, n) or None, passes, flags."""
        torch = self.torch
        n = ins[0].numel()
        arr = (C.c_void_p * 10)(*[t.data_ptr() if t is not None else None for t in ins])
        e = torch.empty(n, dtype=torch.float64, device=self.device)
        u = torch.empty((4, n), dtype=torch.float64, device=self.device)
        pi = torch.empty((5, n), dtype=torch.float64, device=self.device) if with_pi else None
        ps = torch.empty(n, dtype=torch.int32, device=self.device)
        fl = torch.empty(n, dtype=torch.int32, device=self.device)
        uarr = (C.c_void_p * 4)(*[u[m].data_ptr() for m in range(4)])
        parr = C.pointer((C.c_void_p * 5)(*[pi[k].data_ptr() for k in range(5)])) if with_pi else None
        _check(lib().kt_recover_reduced(self.ctx, n, float(tau), arr, C.c_void_p(e.data_ptr()), uarr, parr,
                                        _ptr(ps), _ptr(fl)), self.ctx)
        return e, u, pi, ps, fl

    # ---------------------------------------------- learned inversion start
    def set_inv_start(self, start: int):
        _check(lib().kt_set_inv_start(self.ctx, int(start)), self.ctx)

    def mlp_set(self, params):
        """params: device float32 tensor of KT_MLP_NPARAMS (W1, b1, W2, b2, W3, b3)."""
        assert params.dtype == self.torch.float32 and params.numel() == KT_MLP_NPARAMS
        params = params.contiguous()
        _check(lib().kt_mlp_set(self.ctx, _ptr(params), KT_MLP_NPARAMS), self.ctx)
        self.torch.cuda.synchronize(self.device)

    def mlp_get(self):
        out = self.torch.empty(KT_MLP_NPARAMS, dtype=self.torch.float32, device=self.device)
        _check(lib().kt_mlp_get(self.ctx, _ptr(out), KT_MLP_NPARAMS), self.ctx)
        return out

    def mlp_features(self, ins, tau: float, e=None, u=None):
        """ins: 9 device float64 tensors (n,); e (n,), u (4, n) optional -> x (11, n)[, y (4, n)]."""
        torch = self.torch
        n = ins[0].numel()
        arr = (C.c_void_p * 9)(*[t.data_ptr() if t is not None else None for t in ins])
        x = torch.empty((11, n), dtype=torch.float32, device=self.device)
        y = torch.empty((4, n), dtype=torch.float32, device=self.device) if e is not None else None
        uarr = (C.c_void_p * 4)(*[u[m].data_ptr() for m in range(4)]) if u is not None else None
        _check(lib().kt_mlp_features(self.ctx, n, float(tau), arr, _ptr(e),
                                     C.cast(uarr, C.c_void_p) if uarr is not None else None,
                                     _ptr(x), _ptr(y)), self.ctx)
        return (x, y) if y is not None else x

    def mlp_fwd(self, x, keep_act=False):
        """x (11, n) float32 -> y (4, n)[, act (128, n)]."""
        torch = self.torch
        n = x.shape[1]
        y = torch.empty((4, n), dtype=torch.float32, device=self.device)
        act = torch.empty((128, n), dtype=torch.float32, device=self.device) if keep_act else None
        _check(lib().kt_mlp_fwd(self.ctx, n, _ptr(x.contiguous()), _ptr(y), _ptr(act)), self.ctx)
        return (y, act) if keep_act else y

    def mlp_y0(self, x):
        """x (11, n) float32 -> y_0 (n,): the matrix-core inference of the recoveries."""
        torch = self.torch
        n = x.shape[1]
        y0 = torch.empty((n,), dtype=torch.float32, device=self.device)
        _check(lib().kt_mlp_y0(self.ctx, n, _ptr(x.contiguous()), _ptr(y0)), self.ctx)
        return y0

    def mlp_loss(self, y, t, w=None):
        """-> (loss device float64 scalar tensor, dy (4, n)); w: 4 output weights."""
        torch = self.torch
        n = y.shape[1]
        dy = torch.empty_like(y)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        wp = (C.c_float * 4)(*w) if w is not None else None
        _check(lib().kt_mlp_loss(self.ctx, n, _ptr(y.contiguous()), _ptr(t.contiguous()), wp,
                                 _ptr(dy), _ptr(loss)), self.ctx)
        return loss, dy

    def mlp_bwd(self, x, act, dy):
        grad = self.torch.empty(KT_MLP_NPARAMS, dtype=self.torch.float32, device=self.device)
        _check(lib().kt_mlp_bwd(self.ctx, x.shape[1], _ptr(x.contiguous()), _ptr(act.contiguous()),
                                _ptr(dy.contiguous()), _ptr(grad)), self.ctx)
        return grad

    def mlp_adam(self, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        _check(lib().kt_mlp_adam(self.ctx, _ptr(grad), lr, b1, b2, eps, int(t)), self.ctx)

    def profile(self, on, classes=None):
        """Time the launches of kt_step per kernel class: every class when on is
        true, only the named classes (of PROFILE_CLASSES) when given."""
        mask = 0
        if on:
            names = PROFILE_CLASSES if classes is None else classes
            for n in names:
                mask |= 1 << PROFILE_CLASSES.index(n)
        _check(lib().kt_profile_enable(self.ctx, mask), self.ctx)

    def profile_read(self) -> dict:
        """Summed kernel times (ms) and launch counts per class since the last read."""
        p = KtProfile()
        _check(lib().kt_profile_read(self.ctx, C.byref(p)), self.ctx)
        out = {}
        for k, name in enumerate(PROFILE_CLASSES):
            out[name + "_ms"] = p.ms[k]
            out[name + "_launches"] = p.launches[k]
        return out

    def close(self):
        if getattr(self, "ctx", None):
            lib().kt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several events advanced together (one launch per kernel over all
    events, one step replayed as a hipGraph).

    events: list of (grid, config, prims) sharing the EOS, coordinates,
    precision, tau0 and dtau.
    """

    def __init__(self, events, eos, tau0=None, device="cuda:0", workspace=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.grids = [g for g, _, _ in events]
        n = len(events)
        if tau0 is None:
            tau0 = events[0][2].tau0
        self.params = (KtParams * n)(*[make_params(g, cfg, tau0) for g, cfg, _ in events])
        self.eos_host = EosHost(eos)
        L = lib()
        nbytes = int(L.kt_batch_workspace_bytes(self.params, n, C.byref(self.eos_host.c)))
        if nbytes == 0:
            raise KtError(KT_E_ARG, "invalid batch parameters")
        with torch.cuda.device(self.device):
            # workspace: a caller's uint8 device tensor of at least kt_batch_workspace_bytes
            # (its contents are not assumed), else a new one
            if workspace is not None:
                assert workspace.dtype == torch.uint8 and workspace.numel() >= nbytes
                self.ws = workspace
            else:
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            keep = []
            states = (KtInitState * n)(*[_init_state(torch, self.device, g, pr, None, None, keep)
                                         for g, _, pr in events])
            stream = torch.cuda.current_stream(self.device).cuda_stream
            b = C.c_void_p()
            st = L.kt_batch_init(self.params, n, C.byref(self.eos_host.c), states,
                                 C.c_void_p(self.ws.data_ptr()), nbytes, C.c_void_p(stream), C.byref(b))
            if st != KT_OK:
                raise KtError(st, L.kt_batch_last_error(None).decode(errors="replace"))
            self.b = b
            del keep
        self.n = n

    def _check(self, st):
        if st != KT_OK:
            raise KtError(st, lib().kt_batch_last_error(self.b).decode(errors="replace"))

    def step(self, n: int = 1):
        self._check(lib().kt_batch_step(self.b, int(n)))
        return self

    def tune(self):
        """Autotune the flux block per grid shape; returns (eta planes, block width in x)
        per event."""
        kc = (C.c_int32 * self.n)()
        tile = (C.c_int32 * self.n)()
        self._check(lib().kt_batch_tune(self.b, kc, tile))
        return list(zip(kc, tile))

    def set_flux_blocks(self, blocks):
        """blocks: (eta planes, block width in x) per event, as tune() returns."""
        kc = (C.c_int32 * self.n)(*[int(b[0]) for b in blocks])
        tile = (C.c_int32 * self.n)(*[int(b[1]) for b in blocks])
        self._check(lib().kt_batch_set_flux_blocks(self.b, kc, tile))

    def observables(self, event: int) -> dict:
        o = KtObs()
        self._check(lib().kt_batch_observables(self.b, int(event), C.byref(o), None))
        return o.as_dict()

    def fields(self, event: int, which=("e", "u", "q", "u_prev")) -> dict:
        torch = self.torch
        shape = self.grids[event].shape
        out = {}
        f = KtFields()
        if "e" in which:
            out["e"] = torch.empty(shape, dtype=torch.float64, device=self.device)
            f.e = out["e"].data_ptr()
        for key, n, arr in (("u", 4, f.u), ("u_prev", 4, f.u_prev), ("q", NQ, f.q)):
            if key in which:
                out[key] = torch.empty((n,) + shape, dtype=torch.float64, device=self.device)
                for m in range(n):
                    arr[m] = out[key][m].data_ptr()
        self._check(lib().kt_batch_observables(self.b, int(event), None, C.byref(f)))
        return out

    def close(self):
        if getattr(self, "b", None):
            lib().kt_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
