"""Runs to freeze-out (max T below 155 MeV, Sec. 7): the full 128^3 viscous
hot-spot event in FP64, mixed precision and the reduced state, and the
48-event batch in mixed precision.  No non-finite value, no bisection
fallback, the flow normalised and, in the reduced state, the shear stress
transverse and traceless to rounding (Sec. 2.4) over the whole evolution; the
three states of the 128^3 event end within the differences their arithmetic
allows.  (Properties that hold at any size; the oracle is compared at this
size for 200 steps elsewhere.)"""
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


def test_batch_of_48_events_to_freezeout(kt):
    """The 48 hot-spot events on uneven grids (52.95 M cells, mixed-precision
    state, one launch per kernel for all events, graph-replayed) advanced
    until every event's max T is below 155 MeV: no non-finite value and no
    bisection fallback in any event, the flow normalised and the CFL number
    below one throughout."""
    evs = I.workload_batch()
    T_f = 0.155 / I.HBARC
    b = kt.Batch([(e.grid, e.config, e.prims) for e in evs], evs[0].eos, device="cuda:0")
    b.tune()
    n = len(evs)
    del evs
    done = 0
    for chunk in range(12):
        b.step(100)
        done += 100
        obs = [b.observables(k) for k in range(n)]
        frozen = sum(o["T_max"] < T_f for o in obs)
        print("batch: %d steps, %d of %d events below T_f, max T %.4f GeV" % (
            done, frozen, n, max(o["T_max"] for o in obs) * I.HBARC), flush=True)
        for o in obs:
            assert o["n_nan"] == 0 and o["n_fallback"] == 0 and o["n_fallback_faces"] == 0
            assert o["norm_err"] < 1e-12 and o["cfl"] < 1.0
        if frozen == n:
            break
    b.close()
    assert frozen == n and done <= 1000
