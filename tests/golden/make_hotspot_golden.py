"""Write oracle reference samples for the 128^3 non-conformal viscous hot-spot event.

Runs the FP64 CPU oracle (and nothing else) from the seeded initial state for
200 Heun steps and stores e, u^mu and the 15 evolved components at a seeded
sample of cells after 50, 100 and 200 steps.

It also measures how the event amplifies rounding-sized differences: the same
oracle is run twice more from initial energy densities perturbed in every
cell, once by one FP64 ulp (e -> nextafter(e, inf)) and once by a relative
2^-24 (the size of an FP32 rounding).  The spread between the perturbed and
the unperturbed runs over all cells (dense cells, median, fraction above
1e-9, largest) is stored with the samples; the parity bars of the GPU tests
at 200 steps are set from it.

The file records the SHA-256 of the oracle source that defines the step
(``oracle_sha``: the source above its diagnostics marker); the GPU test
refuses samples made with another oracle.
Usage (about an hour on 8 cores):

    python tests/golden/make_hotspot_golden.py [out.npz]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1608_06577_amd import inputs as I  # noqa: E402

SNAP_STEPS = (50, 100, 200)
ORACLE_SOURCE = os.path.join(ROOT, "oracle", "kt_oracle.c")


STEP_MARKER = b"/* Diagnostics.  Everything above this line defines the step"


def oracle_sha() -> np.ndarray:
    """SHA-256 of the part of the oracle source that defines the step (all of
    it above the diagnostics marker)."""
    src = open(ORACLE_SOURCE, "rb").read()
    cut = src.find(STEP_MARKER)
    assert cut > 0, "diagnostics marker missing from the oracle source"
    return np.frombuffer(hashlib.sha256(src[:cut]).digest(), np.uint8)


def sample_cells(e0: np.ndarray, n_uniform=1536, n_hot=512, seed=2024) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = e0.ravel()
    uni = rng.choice(flat.size, n_uniform, replace=False)
    hot_pool = np.flatnonzero(flat > 0.1 * flat.max())
    hot = rng.choice(hot_pool, n_hot, replace=False)
    return np.unique(np.concatenate([uni, hot]))


def spread(ref, other, tau):
    """Relative differences of e and u between two oracle runs over all cells
    (e: |de| / max(e, 1e-6 e_max); u: |du^mu| / u^tau with u^eta times tau)."""
    emax = ref.e.max()
    de = np.abs(other.e - ref.e) / np.maximum(ref.e, 1e-6 * emax)
    du = np.max(np.abs(other.u - ref.u) * np.array([1, 1, 1, tau]) / ref.u[:, :1], axis=1)
    d = np.maximum(de, du)
    dense = ref.e > 1e-3 * emax
    return dict(max=float(d.max()), dense_max=float(d[dense].max()), median=float(np.median(d)),
                frac_above_1e9=float(np.mean(d > 1e-9)), frac_above_1e7=float(np.mean(d > 1e-7)),
                dense_cells=int(dense.sum()))


def main(out):
    w = I.workload_hotspot()
    phys = oracle.Physics.from_config(w.grid, w.config)
    sim = oracle.Simulation.from_primitives(phys, w.eos, w.prims)
    perturbed = {}
    for name, e0 in (("ulp", np.nextafter(w.prims.e, np.inf)),
                     ("fp32", w.prims.e * (1.0 + 2.0 ** -24))):
        p = I.Primitives(w.prims.grid, w.prims.tau0, e0, w.prims.u, w.prims.pi, w.prims.Pi)
        perturbed[name] = oracle.Simulation.from_primitives(phys, w.eos, p)
    idx = sample_cells(w.prims.e)
    data = dict(idx=idx, input_sha=np.frombuffer(
        hashlib.sha256(np.ascontiguousarray(w.prims.e).tobytes()).digest(), np.uint8),
        oracle_sha=oracle_sha())
    spreads = {}
    t0 = time.time()
    done = 0
    for s in SNAP_STEPS:
        sim.step(s - done)
        for p in perturbed.values():
            p.step(s - done)
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
        spreads[s] = {name: spread(sim, p, sim.tau) for name, p in perturbed.items()}
        print("step %d tau %.3f emax %.6g umax %.4g  %.0fs  spread %s" % (
            s, sim.tau, sim.e.max(), sim.u[:, 0].max(), time.time() - t0, json.dumps(spreads[s])),
            flush=True)
    data["spread_json"] = np.frombuffer(json.dumps(spreads).encode(), np.uint8)
    np.savez_compressed(out, **data)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__),
                                                            "hotspot_128_fp64.npz"))
