"""The inversion's bisection fallback (Sec. 3.2 leaves failure handling open;
reading: bisection on [e_floor, E] to the Newton tolerance when Newton has not
converged within newton_max iterations), forced by newton_max = 1 so that
every state whose conformal start is not already within the tolerance takes
it: the standalone inversion and whole steps (cells and face states) against
the oracle with the same newton_max."""
import numpy as np
import pytest

import oracle
from paper_1608_06577_amd import inputs as I

from tests.test_gpu_parity import e_err, u_err

pytestmark = pytest.mark.gpu
F_FALLBACK = 4


@pytest.fixture(scope="module")
def kt():
    import torch
    assert torch.cuda.is_available()
    from paper_1608_06577_amd import kt as K
    K.lib()
    return K


def test_forced_fallback_inversion_matches_oracle(kt):
    import torch
    from tests.test_oracle_algebra import pack_pi, random_state
    tau = 0.9
    eos = I.eos_c1_table()
    w = I.workload_hotspot(nx=4, ny=4, neta=4)
    cfg = dict(w.config, newton_max=1)
    phys = oracle.Physics.from_config(w.grid, cfg)
    e, u, pi, Pi = random_state(tau, 3000, u_scale=1.5)
    q = oracle.tmunu(phys, eos, tau, e, u, pack_pi(pi), Pi)
    eo, uo, ito, flo = oracle.recover(phys, eos, tau, q)
    gpu = kt.Solver(w.grid, cfg, eos, w.prims)
    ins = [torch.tensor(q[:, k], device="cuda") for k in (0, 1, 2, 3, 4, 5, 6, 7, 14)]
    eg, ug, itg, flg = gpu.recover(ins, tau)
    eg, ug, flg = eg.cpu().numpy(), ug.cpu().numpy().T, flg.cpu().numpy()
    fb = (flo & F_FALLBACK) != 0
    print("forced fallback: %d of %d states bisected" % (fb.sum(), len(fb)), flush=True)
    assert fb.mean() > 0.5
    assert np.array_equal(flg, flo)
    # bisection stops at |f| <= tol E or an interval of 4e-16 e: the two sides
    # evaluate p(e) with different rounding, so a comparison near the root can
    # go either way within that tolerance
    assert np.max(np.abs(eg - eo) / eo) < 1e-11
    assert np.max(np.abs(ug - uo) / uo[:, :1]) < 1e-11
    # and the result is the root Newton finds, within the bisection's stopping
    # rule |f| <= 1e-12 E (|de| = |f| / f', f' = 1 - M^2 c_s^2 / (E + P)^2 <= 1)
    en, _, _, _ = oracle.recover(oracle.Physics.from_config(w.grid, dict(w.config)), eos, tau, q)
    E = q[:, 0] - q[:, 4]
    assert np.max(np.abs(eg - en) / E) < 1e-10


def test_forced_fallback_steps_match_oracle(kt):
    """Five steps of a small hot-spot event with newton_max = 1: every cell and
    face state that the conformal start does not solve is bisected."""
    w = I.workload_hotspot(nx=24, ny=20, neta=8, dx=0.5, deta=0.6, n_hot=20, seed=12)
    cfg = dict(w.config, newton_max=1)
    phys = oracle.Physics.from_config(w.grid, cfg)
    sim = oracle.Simulation.from_primitives(phys, w.eos, w.prims)
    gpu = kt.Solver(w.grid, cfg, w.eos, w.prims)
    sim.step(5)
    gpu.step(5)
    f = {k: v.cpu().numpy() for k, v in gpu.fields().items()}
    r = sim.fields()
    obs = gpu.observables()
    print("forced fallback steps: cells bisected %d of %d, face states %d of %d; e %.2e u %.2e" % (
        obs["n_fallback"], obs["n_recover_cells"], obs["n_fallback_faces"], obs["n_recover_faces"],
        e_err(f["e"], r["e"]), u_err(f["u"], r["u"], sim.tau)), flush=True)
    assert obs["n_fallback"] > 0 and obs["n_fallback_faces"] > 0
    assert obs["n_fallback"] == sim.stats.n_fallback
    assert e_err(f["e"], r["e"]) <= 1e-9 and u_err(f["u"], r["u"], sim.tau) <= 1e-9
