"""kt_init_static (the allocation-free kt_init whose workspace is the library's
static per-GPU array) against kt_init with a caller-owned workspace: two
contexts in a row on the same GPU, the second on a smaller grid, each stepped
and compared field by field with a kt_init context on the same input.  The
kernels are the same, so the fields must agree bit for bit; the oracle is not
needed (kt_init's path is compared with it in test_gpu_parity.py)."""
import numpy as np
import pytest

from paper_1608_06577_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kt():
    import torch
    assert torch.cuda.is_available()
    from paper_1608_06577_amd import kt as K
    K.lib()
    return K


def fields_np(s):
    return {k: v.cpu().numpy() for k, v in s.fields().items()}


def compare(kt, w, n_steps):
    ref = kt.Solver(w.grid, w.config, w.eos, w.prims)
    sta = kt.Solver(w.grid, w.config, w.eos, w.prims, static_workspace=True)
    assert sta.ws is None
    ref.step(n_steps)
    sta.step(n_steps)
    fr, fs = fields_np(ref), fields_np(sta)
    for k in ("e", "u", "q", "u_prev"):
        assert np.array_equal(fr[k], fs[k]), k
    orr, ors = ref.observables(), sta.observables()
    for k in ("energy", "e_max", "newton_iters_cells", "newton_iters_faces", "n_floor", "n_clamp"):
        assert orr[k] == ors[k], (k, orr[k], ors[k])
    ref.close()
    sta.close()
    return fr


def test_static_workspace_matches_kt_init_twice(kt):
    # first call: a hot-spot event with the lattice EOS, bulk and the regulator
    # (32 MiB of workspace); second call: a smaller grid of another shape
    w1 = I.workload_hotspot(nx=56, ny=52, neta=24, dx=0.4, deta=0.5, n_hot=60, seed=3)
    print("no-alloc: first context %s" % (w1.grid.shape,), flush=True)
    f1 = compare(kt, w1, 6)
    w2 = I.workload_hotspot(nx=30, ny=22, neta=9, dx=0.6, deta=0.6, n_hot=20, seed=5)
    print("no-alloc: second context %s" % (w2.grid.shape,), flush=True)
    f2 = compare(kt, w2, 4)
    assert f1["e"].shape != f2["e"].shape
    assert np.isfinite(f2["e"]).all()
