"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/kt.h declares, and rejects invalid arguments before
any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1608_06577_amd import inputs as I
from paper_1608_06577_amd import kt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "kt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kt_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(kt.LIB_PATH):
        from paper_1608_06577_amd import build
        build.build()
    return kt.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n
    assert set(kt.EXPORTS) == set(names)


def good_params():
    g = I.Grid(8, 6, 4, 0.1, 0.1, 0.1)
    return g, I.default_config(eta_s=0.2, zeta_coef=0.1)


def test_workspace_bytes_and_validation(L):
    g, cfg = good_params()
    eos = kt.EosHost(I.eos_c1_table(n=64))
    p = kt.make_params(g, cfg, 0.5)
    n = L.kt_workspace_bytes(C.byref(p), C.byref(eos.c))
    assert n > 43 * 8 * g.ncells and n % 256 == 0
    bad = [("nx", 0), ("dx", 0.0), ("dtau", -1.0), ("theta", 2.5), ("theta", 0.9), ("tau0", 0.0),
           ("e_floor", 0.0), ("m2_delta", 1.0), ("newton_max", 0), ("coords", 7), ("zeta_model", 2),
           ("reduced", 2), ("reduced", -1)]
    for field, val in bad:
        q = kt.make_params(g, cfg, 0.5)
        setattr(q, field, val)
        assert L.kt_workspace_bytes(C.byref(q), C.byref(eos.c)) == 0, field
    q = kt.make_params(g, cfg, 0.5)
    q.zeta_model, q.zeta_tc = 1, 0.0            # the paper's zeta/s(T) needs T_c > 0
    assert L.kt_workspace_bytes(C.byref(q), C.byref(eos.c)) == 0
    q.zeta_tc = 0.2 / I.HBARC
    assert L.kt_workspace_bytes(C.byref(q), C.byref(eos.c)) == n
    small = I.eos_c1_table(n=64)
    small.p = small.p[:1]
    small.cs2 = small.cs2[:1]
    small.T = small.T[:1]
    e1 = kt.EosHost(small)
    assert L.kt_workspace_bytes(C.byref(p), C.byref(e1.c)) == 0


def test_init_rejects_bad_arguments_without_device_work(L):
    g, cfg = good_params()
    eos = kt.EosHost(I.eos_conformal())
    p = kt.make_params(g, cfg, 0.5)
    ctx = C.c_void_p()
    st = kt.KtInitState()
    # null state / workspace
    assert L.kt_init(C.byref(p), C.byref(eos.c), None, None, 0, None, C.byref(ctx)) == kt.KT_E_ARG
    assert b"null" in L.kt_last_error(None)
    # bad grid
    q = kt.make_params(g, cfg, 0.5)
    q.ny = -3
    assert L.kt_init(C.byref(q), C.byref(eos.c), C.byref(st), C.c_void_p(256), 1 << 30, None,
                     C.byref(ctx)) == kt.KT_E_ARG
    assert b"grid" in L.kt_last_error(None)
    # misaligned workspace
    assert L.kt_init(C.byref(p), C.byref(eos.c), C.byref(st), C.c_void_p(8), 1 << 30, None,
                     C.byref(ctx)) == kt.KT_E_ARG
    # neither q nor primitives
    assert L.kt_init(C.byref(p), C.byref(eos.c), C.byref(st), C.c_void_p(4096), 1 << 30, None,
                     C.byref(ctx)) == kt.KT_E_ARG
    # workspace too small
    for c in range(15):
        st.q[c] = 4096
    assert L.kt_init(C.byref(p), C.byref(eos.c), C.byref(st), C.c_void_p(4096), 1024, None,
                     C.byref(ctx)) == kt.KT_E_ALLOC
    # a resumed state (q and e) needs u
    st.e = 4096
    assert L.kt_init(C.byref(p), C.byref(eos.c), C.byref(st), C.c_void_p(4096), 1 << 30, None,
                     C.byref(ctx)) == kt.KT_E_ARG
    assert b"resume" in L.kt_last_error(None)
    st.e = None
    # unknown precision
    q = kt.make_params(g, cfg, 0.5)
    q.precision = 7
    assert L.kt_init(C.byref(q), C.byref(eos.c), C.byref(st), C.c_void_p(4096), 1 << 30, None,
                     C.byref(ctx)) == kt.KT_E_ARG
    assert L.kt_workspace_bytes(C.byref(q), C.byref(eos.c)) == 0
    assert not ctx.value
    # the mixed-precision state needs less workspace: 4 FP64 + 11 FP32 components per q
    q.precision = kt.KT_MIXED
    n_mixed = L.kt_workspace_bytes(C.byref(q), C.byref(eos.c))
    assert 0 < n_mixed < L.kt_workspace_bytes(C.byref(p), C.byref(eos.c))
    # calls on a null context
    assert L.kt_step(None, 1) == kt.KT_E_ARG
    assert L.kt_observables(None, None, None) == kt.KT_E_ARG
    assert L.kt_validity(None, None, None, None, None, None, None, None, None) == kt.KT_E_ARG
    n_done = C.c_int32(-1)
    assert L.kt_run_to_freezeout(None, 0.7, 10, 1, C.byref(n_done)) == kt.KT_E_ARG
    L.kt_destroy(None)
    assert L.kt_status_string(kt.KT_E_ALLOC) == b"workspace too small"


def test_learned_start_entry_points_reject_null_context(L):
    """Argument marshalling of every learned-start entry point and of the
    reduced recovery, nullable arguments given as null: each rejects the null
    context before any device work."""
    vp = C.c_void_p
    arr9 = (vp * 9)()
    u4 = C.cast((vp * 4)(), vp)
    w4 = (C.c_float * 4)(1.0, 0.5, 0.5, 0.5)
    calls = [
        L.kt_set_inv_start(None, kt.KT_START_LEARNED),
        L.kt_mlp_set(None, None, kt.KT_MLP_NPARAMS),
        L.kt_mlp_get(None, None, kt.KT_MLP_NPARAMS),
        L.kt_mlp_features(None, 4, 1.0, arr9, None, None, None, None),
        L.kt_mlp_features(None, 4, 1.0, arr9, None, u4, None, None),
        L.kt_mlp_fwd(None, 4, None, None, None),
        L.kt_mlp_loss(None, 4, None, None, None, None, None),
        L.kt_mlp_loss(None, 4, None, None, w4, None, None),
        L.kt_mlp_bwd(None, 4, None, None, None, None),
        L.kt_mlp_adam(None, None, 1e-3, 0.9, 0.999, 1e-8, 1),
        L.kt_recover_reduced(None, 4, 1.0, (vp * 10)(), None, (vp * 4)(), None, None, None),
    ]
    assert all(c == kt.KT_E_ARG for c in calls), calls
    assert b"null context" in L.kt_last_error(None)


def test_static_init_rejects_grids_beyond_its_array(L):
    """kt_init_static checks the grid against KT_STATIC_WS_BYTES before any
    device work."""
    g = I.Grid(128, 128, 128, 0.16, 0.16, 0.1)
    cfg = I.default_config(eta_s=0.2, zeta_coef=0.1)
    eos = kt.EosHost(I.eos_c1_table(n=64))
    p = kt.make_params(g, cfg, 0.5)
    assert L.kt_workspace_bytes(C.byref(p), C.byref(eos.c)) > 64 << 20
    ctx = C.c_void_p()
    st = kt.KtInitState()
    assert L.kt_init_static(C.byref(p), C.byref(eos.c), C.byref(st), None, C.byref(ctx)) == 2
    assert not ctx.value
    assert b"static workspace" in L.kt_last_error(None)
    p.nx = 0
    assert L.kt_init_static(C.byref(p), C.byref(eos.c), C.byref(st), None, C.byref(ctx)) == 1
