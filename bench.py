"""Benchmark: Heun steps of the 128^3 non-conformal viscous hot-spot event (FP64).

One step is one full Heun step of the KT scheme (two stages, two recoveries)
over the whole 128^3 grid, replayed from a captured hipGraph.  Prints one
JSON line:
  value        cell-updates/s (128^3 cells x steps / seconds), inputs resident in HBM
  roofline     the whole step against HBM: 103 algorithmic values (824 B in FP64) per
               cell and step x cells / the mean step time (HIP events over the timed
               region); traffic: rocprofv3 counter bytes of one step
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same event, on all
               host threads and on one

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-probe]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
METRIC = "cell-updates/s per Heun step (128^3 viscous), % HBM peak; learned vs Newton"
# algorithmic values moved per cell (8 bytes each in FP64):
#   stage 1 reads q^n (15), u^n (4), u^{n-1} (4), e^n (1) and writes q* (15)            = 39
#   stage 2 reads q* (15), u* (4), e* (1), u^n (4), q^n (15) and writes q^{n+1} (15)     = 54
#   the two recoveries write u and e (10)                                              = 10
#   one Heun step moves 103 values (p is recomputed, not stored)
STEP_VALUES = 103
# mixed-precision state: T^{tau mu} (4 of the 15 q components) and u (4) stay 8 bytes,
# the other 11 q components and e are 4 bytes: 492 B per cell and step
STEP_BYTES_MIXED = 492.0
# algorithmic values per cell and launch of each kernel class, averaged over the two stages
# (diagnostics: the per-kernel fractions):
#   flux     reads q (15) and the stage accumulator (15), writes it (15)           = 45
#   sources  reads q (15), u (4), u_prev (4), e, p and, in stage 2, q^n (15);
#            writes 15                                                             = 40 / 55
#   recover  reads q (15), e; writes e, p, u (4) and the 10 regulated pi           = 32
#   faces    reads 9 components of q and e; writes v^-, v^+ of 3 faces (6)         = 16
KERNEL_VALUES = {"flux": 45.0, "sources": 47.5, "recover": 32.0, "faces": 16.0}
# launches of each class per Heun step
LAUNCHES_PER_STEP = {"flux": 2, "sources": 2, "recover": 2, "faces": 2}
# HBM bytes per launch of the FP64 step graph's kernels on this event (mean of the two
# stages' launches of a class), from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by what the
# counters read for a plain device copy (FETCH x 2, WRITE x 1; profiles/); valid for the kernel
# sources and compiler flags whose hash is TRAFFIC_SOURCES (else the traffic is reported as null).
# The flux kernel's traffic depends on its block ("eta planes x cells in x", the block the
# autotuner picks); a block without a measured figure reports null.
TRAFFIC_SOURCES = "2e50fc48d2a6ebf9"
TRAFFIC_BYTES = {"flux": {"2x64": 1306860016, "4x64": 1111773200}, "sources": 1187809024,
                 "faces": 694087392, "recover": 584777640}
KERNEL_NAMES = {"flux": "flux_kernel (KT flux divergence + stage update)",
                "sources": "sources_kernel (App. B sources + stage update)",
                "recover": "recover_kernel (Newton inversion + regulator)",
                "faces": "face_speeds_kernel (inversion of reconstructed face states)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (for counter scaling)")
    ap.add_argument("--n", type=int, default=128, help="grid cells per axis")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-events leg")
    ap.add_argument("--no-lattice", action="store_true", help="skip the lattice-QCD EOS and zeta/s(T) leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start leg")
    ap.add_argument("--no-reduced", action="store_true", help="skip the reduced-state leg")
    ap.add_argument("--flux-block", default=None, metavar="PLANES,CELLS_X",
                    help="flux block of the FP64 step graph (eta planes, cells in x) instead of the autotuner's")
    ap.add_argument("--learn-steps", type=int, default=3000, help="Adam steps of the start network")
    return ap.parse_args()


def kernel_sources_hash():
    """First 16 hex digits of the SHA-256 of the kernel sources, concatenated, and
    of the compiler flags they are built with."""
    import hashlib
    from paper_1608_06577_amd import build
    h = hashlib.sha256()
    for f in ("kt_main.hip", "kt_device.hpp", "kt_mlp.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1608_06577_amd", "csrc", f), "rb").read())
    h.update(" ".join(build.HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def copy_probe():
    import torch
    n = 256 * 1024 * 1024 // 8          # 256 MiB of doubles
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "launches": 3}), flush=True)


def copy_gbs(torch) -> float:
    """Bandwidth of a plain 1 GiB device-to-device copy (bytes read + written / time)."""
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(5):
        y.copy_(x)
    stop.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * n * 8 / (start.elapsed_time(stop) * 1e-3) / 1e9
    del x, y
    return gbs


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s):
    """The FP64 oracle on the host's cores: the mean over up to 3 Heun steps of
    the 128^3 event on all threads, then one step on one thread (the paper's
    serial CPU timings, Tables 980ti_compare and k20M_compare, are one core)."""
    import oracle
    phys = oracle.Physics.from_config(w.grid, w.config)
    n_all = oracle.num_threads()
    t0 = time.perf_counter()
    sim = oracle.Simulation.from_primitives(phys, w.eos, w.prims)
    t_init = time.perf_counter() - t0
    steps = 0
    t1 = time.perf_counter()
    while steps < 1 or (time.perf_counter() - t1 < budget_s and steps < 3):
        sim.step(1)
        steps += 1
    dt = time.perf_counter() - t1
    oracle.set_num_threads(1)
    t2 = time.perf_counter()
    sim.step(1)
    dt1 = time.perf_counter() - t2
    oracle.set_num_threads(n_all)
    return {"value": w.grid.ncells * steps / dt, "unit": "cell-updates/s",
            "cores": n_all, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d Heun step(s) of the same %dx%dx%d event from its initial state on %d "
                      "threads (%.1f s, plus %.1f s initial recovery)" % (
                          steps, w.grid.nx, w.grid.ny, w.grid.neta, n_all, dt, t_init),
            "single_thread": {"value": w.grid.ncells / dt1, "unit": "cell-updates/s", "cores": 1,
                              "sample": "the next Heun step of the same event on 1 thread "
                                        "(%.1f s)" % dt1}}


def time_graph_steps(torch, batch, warmup, steps):
    """Mean time of one replayed step graph (HIP events on the caller's stream,
    which the replays are ordered between)."""
    batch.step(warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    batch.step(steps)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def learned_leg(args, kt, I, torch):
    """Learned inversion start on a 200 x 200 x 96 hot-spot event in mixed
    precision (FP32 state): the start network is trained on the event's own
    states by the library's kernels, then the same steps are timed from the
    same initial state with the plain warm start, the conformal start and the
    learned start.  Every start is polished by the same Newton iteration to the
    same tolerance, so the fields agree to rounding."""
    from paper_1608_06577_amd import learned
    w = I.workload_hotspot(nx=200, ny=200, neta=96, seed=11)
    cfg = dict(w.config)
    cfg["mixed"] = True
    ncell = w.grid.ncells
    print("bench: learned start, %s, mixed precision: training" % "x".join(map(str, w.grid.shape[::-1])),
          file=sys.stderr, flush=True)
    t0 = time.time()
    trainer = kt.Solver(w.grid, cfg, w.eos, w.prims, device="cuda:0")
    trainer.mlp_set(torch.tensor(I.mlp_init_params(0), device="cuda:0"))
    X, T = learned.collect_pairs(trainer, cfg["e_floor"], n_snap=6, steps_between=10, max_pairs=2_000_000)
    n_pairs = X.shape[1]
    losses = learned.train(trainer, X, T, steps=args.learn_steps)
    params = trainer.mlp_get()
    trainer.close()
    del X, T
    torch.cuda.synchronize()
    t_train = time.time() - t0
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out, fields = {}, {}
    for mode, code in (("plain_warm", kt.KT_START_WARM), ("conformal", kt.KT_START_CONFORMAL),
                       ("learned", kt.KT_START_LEARNED)):
        s = kt.Solver(w.grid, cfg, w.eos, w.prims, device="cuda:0")
        if code == kt.KT_START_LEARNED:
            s.mlp_set(params)
        s.set_inv_start(code)
        s.step(args.warmup)
        o0 = s.observables()
        torch.cuda.synchronize()
        start.record()
        s.step(args.steps)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.steps
        o1 = s.observables()
        iters = (o1["newton_iters_cells"] - o0["newton_iters_cells"]) / max(1, o1["n_recover_cells"] - o0["n_recover_cells"])
        fields[mode] = s.fields(("e",))["e"].double()
        out[mode] = {"ms_per_step": ms, "value": ncell / (ms * 1e-3), "newton_iters_per_cell": iters,
                     "n_fallback": o1["n_fallback"]}
        s.close()
        print("bench: learned-start leg, %s start: %.3f ms/step, %.3f Newton iterations per cell"
              % (mode, ms, iters), file=sys.stderr, flush=True)
    ref = fields["plain_warm"]
    dense = ref > 1e-3 * ref.max()
    for mode in ("conformal", "learned"):
        d = (fields[mode] - ref).abs() / ref
        out[mode]["max_rel_diff_e_vs_plain_dense_cells"] = d[dense].max().item()
    out.update({"workload": "hotspot_viscous_200x200x96", "state": "mixed precision",
                "training": {"pairs": int(n_pairs), "adam_steps": args.learn_steps,
                             "loss_first_last": [losses[0], losses[-1]], "seconds": t_train},
                "network": "11-64-64-4 GELU, FP32; start = y_0 * conformal root; Newton polish to 1e-12"})
    return out


def lattice_leg(args, rec, w, ncell, torch, kt, I):
    """The headline event and step count in FP64 with the paper's own physics
    of Sec. 2: the lattice-QCD EOS table and the bulk viscosity zeta/s(T)
    (Eq. zetas, normalisation 1, T_c = 200 MeV) instead of the synthetic EOS
    and zeta/s = 0.1 (1/3 - c_s^2).  Replayed from the step graph."""
    eos_l = I.eos_lattice_table()
    cfg = dict(w.config, zeta_model=1, zeta_coef=1.0, zeta_tc=0.2 / I.HBARC)
    bl = kt.Batch([(w.grid, cfg, w.prims)], eos_l, device="cuda:0")
    bl.tune()
    ms_l = time_graph_steps(torch, bl, args.warmup, args.steps)
    obs_l = bl.observables(0)
    rec["variants"]["lattice_eos"] = {
        "ms_per_step": ms_l, "value": ncell / (ms_l * 1e-3), "state": "FP64",
        "eos": "lattice-QCD trace-anomaly fit, 4096 nodes", "zeta_over_s": "zeta/s(T), T_c = 200 MeV",
        "step_hbm_frac": STEP_VALUES * 8.0 * ncell / (ms_l * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "newton_iters_per_cell": obs_l["newton_iters_cells"] / max(1, obs_l["n_recover_cells"]),
        "n_nan": obs_l["n_nan"]}
    bl.close()
    print("bench: lattice-QCD EOS and zeta/s(T) %.3f ms/step" % ms_l, file=sys.stderr, flush=True)


# algorithmic values per cell and Heun step of the reduced state (T^{tau mu}, five pi
# components and Pi evolved, 3 u components stored, u^tau from u.u = 1; Sec. 2.4):
#   stage 1 reads q^n (10), u^n (3), u^{n-1} (3), e^n (1), writes q* (10), u* (3), e* (1)    = 31
#   stage 2 reads q* (10), u* (3), e* (1), u^n (3), q^n (10), writes q^{n+1} (10), u (3), e (1) = 41
STEP_VALUES_REDUCED = 72


def reduced_leg(args, rec, w, ncell, torch, kt):
    """The headline event and step count with the reduced state (kt_params.reduced):
    the recovery solves for (e, u) and the five dependent pi components by a fixed
    point (one inversion per pass); the flux and stage updates skip those five.
    Replayed from the step graph; per-kernel eager launch times beside it."""
    out = {}
    for mixed in (False, True):
        cfg = dict(w.config, reduced=True, mixed=mixed)
        b = kt.Batch([(w.grid, cfg, w.prims)], w.eos, device="cuda:0")
        b.tune()
        o0 = b.observables(0)
        ms = time_graph_steps(torch, b, args.warmup, args.steps)
        o1 = b.observables(0)
        b.close()
        per, ms_eager, _ = eager_kernel_times(kt, torch, w, cfg, min(args.steps, 10))
        nrec = max(1, o1["n_recover_cells"] - o0["n_recover_cells"])
        out["mixed" if mixed else "fp64"] = {
            "ms_per_step": ms, "value": ncell / (ms * 1e-3),
            "state": "T^{tau mu} and u FP64; pi, Pi, e, p FP32" if mixed else "FP64",
            "step_hbm_frac_of_reduced_balg": (None if mixed else
                                              STEP_VALUES_REDUCED * 8.0 * ncell / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)),
            "fixed_point_passes_per_recovery": (o1["fp_passes"] - o0["fp_passes"]) / nrec,
            "newton_iters_per_recovery": (o1["newton_iters_cells"] - o0["newton_iters_cells"]) / nrec,
            "recoveries_not_converged": o1["fp_not_converged"] - o0["fp_not_converged"],
            "eager_ms_per_step": ms_eager, "per_kernel_launch_ms": per, "n_nan": o1["n_nan"]}
        print("bench: reduced state%s %.3f ms/step, %.2f fixed-point passes per recovery" % (
            " (mixed)" if mixed else "", ms, out["mixed" if mixed else "fp64"]["fixed_point_passes_per_recovery"]),
            file=sys.stderr, flush=True)
    out["algorithmic_values_per_cell_step"] = STEP_VALUES_REDUCED
    rec["variants"]["reduced_state"] = out


def eager_kernel_times(kt, torch, w, cfg, n_steps):
    """Per-launch times of the four kernel classes of the eager step (HIP events
    around each launch on the library's stream; outside the timed region), and
    the eager step time."""
    s = kt.Solver(w.grid, cfg, w.eos, w.prims, device="cuda:0")
    s.step(2)
    s.profile(True)
    s.step(n_steps)
    prof = s.profile_read()
    s.profile(False)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    s.step(n_steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / n_steps
    obs = s.observables()
    s.close()
    per = {k: prof[k + "_ms"] / max(1, prof[k + "_launches"]) for k in kt.PROFILE_CLASSES}
    return per, ms, obs


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr, flush=True)
        sys.exit(2)
    import torch
    if args.copy_probe:
        copy_probe()
        return
    from paper_1608_06577_amd import inputs as I
    from paper_1608_06577_amd import kt

    w = I.workload_hotspot(nx=args.n, ny=args.n, neta=args.n)
    ncell = w.grid.ncells
    # the headline: the FP64 step replayed from its captured graph (a batch of
    # one event: the same kernels per cell, tau kept on the device)
    print("bench: %s, FP64, step graph, warmup %d steps" % (w.name, args.warmup), file=sys.stderr, flush=True)
    b = kt.Batch([(w.grid, w.config, w.prims)], w.eos, device="cuda:0")
    if args.flux_block:
        blocks = [tuple(int(v) for v in args.flux_block.split(","))]
        b.set_flux_blocks(blocks)
    else:
        blocks = b.tune()
    ms = time_graph_steps(torch, b, args.warmup, args.steps)
    obs = b.observables(0)
    b.close()
    value = ncell / (ms * 1e-3)
    step_bytes = STEP_VALUES * 8.0 * ncell
    achieved = step_bytes / (ms * 1e-3) / 1e9
    print("bench: timed %d graph steps, %.3f ms/step, %.3g cell-updates/s, %.3f of the HBM roofline"
          % (args.steps, ms, value, achieved / HBM_PEAK_GBS), file=sys.stderr, flush=True)
    # diagnostics outside the timed region: per-kernel times of the eager step
    per, ms_eager, _ = eager_kernel_times(kt, torch, w, w.config, min(args.steps, 10))
    print("bench: eager step %.3f ms; per launch: %s" % (
        ms_eager, ", ".join("%s %.3f ms" % kv for kv in per.items())), file=sys.stderr, flush=True)
    cgbs = copy_gbs(torch)
    traffic = None
    flux_traffic = TRAFFIC_BYTES["flux"].get("%dx%d" % tuple(blocks[0]))
    if kernel_sources_hash() == TRAFFIC_SOURCES and flux_traffic:
        traffic = sum((flux_traffic if k == "flux" else TRAFFIC_BYTES[k]) * LAUNCHES_PER_STEP[k]
                      for k in TRAFFIC_BYTES)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "one Heun step (the captured graph of its launches)",
            "bytes_per_launch": step_bytes, "mean_launch_ms": ms,
            "traffic_over_algorithmic": None if traffic is None else traffic / step_bytes,
            "copy_kernel_gbs": cgbs,
            "per_kernel": {k: {"launch_ms": per[k], "launches_per_step": LAUNCHES_PER_STEP[k],
                               "frac": 8.0 * ncell * KERNEL_VALUES[k] / (per[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                           for k in kt.PROFILE_CLASSES}}
    rec = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.grid.nx, w.grid.ny, w.grid.neta],
                   "dx_fm": w.grid.dx, "deta": w.grid.deta, "tau0": w.tau0,
                   "dtau": w.config["dtau"], "eta_over_s": w.config["eta_s"],
                   "zeta_over_s": "0.1 (1/3 - c_s^2)", "eos": "tabulated, 4096 nodes",
                   "precision": "fp64", "inversion_start": "conformal closed-form root",
                   "flux_block": {"eta_planes": blocks[0][0], "cells_x": blocks[0][1],
                                  "cells_y": 256 // blocks[0][1]},
                   "paper_context_ms_per_step": {"gtx980ti_fp32_128cube_table": 244.45,
                                                 "gtx980ti_program_summary": 38400.0}},
        "roofline": roof,
        "diagnostics": dict({k: obs[k] for k in ("tau", "n_nan", "n_floor", "n_clamp", "n_fallback",
                                                 "n_fallback_faces", "e_max", "cfl")},
                            eager_ms_per_step=ms_eager,
                            newton_iters_per_cell=obs["newton_iters_cells"] / max(1, obs["n_recover_cells"]),
                            newton_iters_per_face_state=obs["newton_iters_faces"] / max(1, obs["n_recover_faces"])),
    }
    # the mixed-precision state on the same event and step count (reported beside the FP64 line)
    cfg_m = dict(w.config)
    cfg_m["mixed"] = True
    bm = kt.Batch([(w.grid, cfg_m, w.prims)], w.eos, device="cuda:0")
    bm.tune()
    ms_m = time_graph_steps(torch, bm, args.warmup, args.steps)
    bm.close()
    per_m, ms_m_eager, _ = eager_kernel_times(kt, torch, w, cfg_m, min(args.steps, 10))
    rec["variants"] = {"mixed_precision": {
        "ms_per_step": ms_m, "value": ncell / (ms_m * 1e-3),
        "step_hbm_frac": STEP_BYTES_MIXED * ncell / (ms_m * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "eager_ms_per_step": ms_m_eager, "per_kernel_launch_ms": per_m,
        "state": "T^{tau mu} and u FP64; pi, Pi, e, p, face speeds FP32; inversion FP64"}}
    print("bench: mixed precision %.3f ms/step (eager %.3f)" % (ms_m, ms_m_eager), file=sys.stderr, flush=True)
    # the same event and step count, FP64, with the lattice-QCD EOS table (Sec. 2)
    if not args.no_lattice:
        lattice_leg(args, rec, w, ncell, torch, kt, I)
    if not args.no_reduced:
        reduced_leg(args, rec, w, ncell, torch, kt)
    if not args.no_batch:
        # 48 hot-spot events on uneven grids, FP32 state, one launch per kernel for all
        # events, one step replayed as a hipGraph, tiling autotuned
        evs = I.workload_batch()
        ncb = sum(e.grid.ncells for e in evs)
        batch = kt.Batch([(e.grid, e.config, e.prims) for e in evs], evs[0].eos, device="cuda:0")
        shapes_b = [tuple(e.grid.shape[::-1]) for e in evs]
        del evs
        blocks_b = batch.tune()
        ms_b = time_graph_steps(torch, batch, args.warmup, args.steps)
        rec["variants"]["batch_48_events"] = {
            "ms_per_step": ms_b, "value": ncb / (ms_b * 1e-3), "cells": ncb,
            "step_hbm_frac": STEP_BYTES_MIXED * ncb / (ms_b * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "shapes": [list(s) for s in I.BATCH_SHAPES],
            "flux_block_per_shape": {"x".join(map(str, sh)): {"eta_planes": bl[0], "cells_x": bl[1],
                                                              "cells_y": 256 // bl[1]}
                                     for sh, bl in zip(shapes_b, blocks_b)},
            "state": "mixed precision; all events per launch; step replayed as a hipGraph"}
        batch.close()
        print("bench: batch of 48 events %.3f ms/step (%.3g cell-updates/s)" % (ms_b, ncb / (ms_b * 1e-3)),
              file=sys.stderr, flush=True)
    if not args.no_learned:
        rec["variants"]["learned_start"] = learned_leg(args, kt, I, torch)
    if not args.no_cpu:
        print("bench: CPU oracle baseline (bounded sample)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
