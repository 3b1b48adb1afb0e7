"""The full 128^3 viscous hot-spot event run to freeze-out (max T below
155 MeV, Sec. 7) in FP64, mixed precision and the reduced state: no
non-finite value, no bisection fallback, the flow normalised and the shear
stress transverse and traceless to rounding (Sec. 2.4) over the whole
evolution, and the three states ending within the differences their
arithmetic allows.  (Properties that hold at any size; the oracle is
compared at this size for 200 steps elsewhere.)"""
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


def test_hotspot_128_to_freezeout(kt):
    import torch
    w = I.workload_hotspot()
    T_f = 0.155 / I.HBARC
    res = {}
    for mode in ("fp64", "mixed", "reduced"):
        cfg = dict(w.config, mixed=mode == "mixed", reduced=mode == "reduced")
        s = kt.Solver(w.grid, cfg, w.eos, w.prims)
        n = s.run_to_freezeout(T_f, 4000, 20)
        o = s.observables()
        print("%s: freeze-out after %d steps, tau %.2f fm, T_max %.4f GeV, e_max %.3g, fallbacks %d/%d, "
              "|u.u - 1| %.1e, pi.u %.1e, pi trace %.1e, cfl %.3f" % (
                  mode, n, o["tau"], o["T_max"] * I.HBARC, o["e_max"], o["n_fallback"], o["n_fallback_faces"],
                  o["norm_err"], o["pi_transverse"], o["pi_trace"], o["cfl"]), flush=True)
        assert 0 < n < 4000 and o["T_max"] < T_f
        assert o["n_nan"] == 0 and o["n_fallback"] == 0 and o["n_fallback_faces"] == 0
        assert o["norm_err"] < 1e-12 and o["cfl"] < 1.0
        if mode == "reduced":
            assert o["pi_transverse"] < 1e-10 and o["pi_trace"] < 1e-10
        res[mode] = (n, s.fields(("e",))["e"])
        s.close()
    # the FP64 and reduced states freeze out within a check interval of each
    # other, mixed precision likewise
    assert abs(res["mixed"][0] - res["fp64"][0]) <= 20 and abs(res["reduced"][0] - res["fp64"][0]) <= 40
