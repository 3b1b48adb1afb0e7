"""Write oracle reference samples for the 128^3 non-conformal viscous hot-spot event.

Runs the FP64 CPU oracle (and nothing else) from the seeded initial state for
200 Heun steps and stores e, u^mu and the 15 evolved components at a seeded
sample of cells after 50, 100 and 200 steps.  Usage (about half an hour on 8
cores):

    python tests/golden/make_hotspot_golden.py [out.npz]
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1608_06577_amd import inputs as I  # noqa: E402

SNAP_STEPS = (50, 100, 200)


def sample_cells(e0: np.ndarray, n_uniform=1536, n_hot=512, seed=2024) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = e0.ravel()
    uni = rng.choice(flat.size, n_uniform, replace=False)
    hot_pool = np.flatnonzero(flat > 0.1 * flat.max())
    hot = rng.choice(hot_pool, n_hot, replace=False)
    return np.unique(np.concatenate([uni, hot]))


def main(out):
    w = I.workload_hotspot()
    phys = oracle.Physics.from_config(w.grid, w.config)
    sim = oracle.Simulation.from_primitives(phys, w.eos, w.prims)
    idx = sample_cells(w.prims.e)
    data = dict(idx=idx, input_sha=np.frombuffer(
        hashlib.sha256(np.ascontiguousarray(w.prims.e).tobytes()).digest(), np.uint8))
    t0 = time.time()
    done = 0
    for s in SNAP_STEPS:
        sim.step(s - done)
        done = s
        data["tau_%d" % s] = np.float64(sim.tau)
        data["e_%d" % s] = sim.e[idx].copy()
        data["u_%d" % s] = sim.u[idx].copy()
        data["q_%d" % s] = sim.q[idx].copy()
        data["Ttt_sum_%d" % s] = np.float64(sim.q[:, 0].sum())
        data["emax_%d" % s] = np.float64(sim.e.max())
        data["stats_%d" % s] = np.array([sim.stats.newton_iters, sim.stats.n_recover,
                                         sim.stats.n_floor, sim.stats.n_clamp,
                                         sim.stats.n_fallback], np.int64)
        print("step %d tau %.3f emax %.6g umax %.4g  %.0fs" % (s, sim.tau, sim.e.max(),
              sim.u[:, 0].max(), time.time() - t0), flush=True)
    np.savez_compressed(out, **data)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__),
                                                            "hotspot_128_fp64.npz"))
