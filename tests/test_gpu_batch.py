"""Batches of events (kt_batch_*) against separate contexts and the oracle.

One launch per kernel covers every event and one step is replayed as a
hipGraph; the arithmetic per cell is that of a single context, so the
results must agree bit for bit, after any number of replays, with eager work
in between, and after the autotuner changes the flux tiling."""
import numpy as np
import pytest

import oracle
from paper_1608_06577_amd import inputs as I

from tests.test_gpu_parity import e_err, u_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kt():
    import torch
    assert torch.cuda.is_available()
    from paper_1608_06577_amd import kt as K
    K.lib()
    return K


def events(mixed=False):
    """Uneven grids (tails in x, y and eta) with different hot-spot draws."""
    out = []
    for (nx, ny, ne, hot, seed) in ((40, 36, 12, 30, 11), (24, 20, 8, 20, 12), (71, 17, 5, 40, 13)):
        w = I.workload_hotspot(nx=nx, ny=ny, neta=ne, dx=0.5, deta=0.6, n_hot=hot, seed=seed)
        cfg = dict(w.config)
        if mixed:
            cfg["mixed"] = True
        out.append((w.grid, cfg, w.prims))
    return out, w.eos


def same(a, b):
    return all(np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()) for k in a)


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_equals_separate_contexts(kt, mixed):
    evs, eos = events(mixed)
    batch = kt.Batch(evs, eos)
    singles = [kt.Solver(g, cfg, eos, pr) for g, cfg, pr in evs]
    # replays of the captured step, with eager observables in between
    for n in (1, 3, 4):
        batch.step(n)
        for s in singles:
            s.step(n)
        for k, s in enumerate(singles):
            assert same(batch.fields(k), s.fields()), (mixed, n, k)
            ob, os_ = batch.observables(k), s.observables()
            assert ob["step"] == os_["step"] and ob["tau"] == os_["tau"]
            assert ob["newton_iters_cells"] == os_["newton_iters_cells"]
            assert ob["newton_iters_faces"] == os_["newton_iters_faces"]


def test_batch_tuning_keeps_results(kt):
    evs, eos = events()
    batch = kt.Batch(evs, eos)
    singles = [kt.Solver(g, cfg, eos, pr) for g, cfg, pr in evs]
    batch.step(2)
    blocks = batch.tune()
    print("autotuned flux blocks (eta planes, x width) per event:", blocks, flush=True)
    assert all(k in (2, 4) and t in (64, 32, 16) for k, t in blocks) and len({k for k, _ in blocks}) == 1
    batch.step(5)
    for s in singles:
        s.step(7)
    for k, s in enumerate(singles):
        assert same(batch.fields(k), s.fields()), k


def test_every_flux_block_gives_the_same_fields(kt):
    """The flux block shapes (64 x 4, 32 x 8, 16 x 16 cells, set per event; 2 or
    4 eta planes) against separate contexts: equal bit for bit."""
    evs, eos = events()
    singles = [kt.Solver(g, cfg, eos, pr) for g, cfg, pr in evs]
    for s in singles:
        s.step(3)
    ref = [s.fields() for s in singles]
    n = len(evs)
    tiles = (64, 32, 16)
    for t0 in range(3):
        for kc in (2, 4):
            # a different width for every event: the events' blocks interleave in each launch
            blocks = [(kc, tiles[(t0 + e) % 3]) for e in range(n)]
            batch = kt.Batch(evs, eos)
            batch.set_flux_blocks(blocks)
            batch.step(3)
            for k in range(n):
                assert same(batch.fields(k), ref[k]), (blocks, k)
            batch.close()
    batch = kt.Batch(evs, eos)
    with pytest.raises(kt.KtError):
        batch.set_flux_blocks([(4, 48)] * n)
    with pytest.raises(kt.KtError):
        batch.set_flux_blocks([(1, 64)] * n)
    with pytest.raises(kt.KtError):
        batch.set_flux_blocks([(2, 64)] + [(4, 64)] * (n - 1))
    batch.close()


def test_batch_matches_oracle(kt):
    """The batch against the FP64 oracle (10 steps, every event)."""
    evs, eos = events()
    batch = kt.Batch(evs, eos)
    batch.step(10)
    for k, (g, cfg, pr) in enumerate(evs):
        phys = oracle.Physics.from_config(g, cfg)
        sim = oracle.Simulation.from_primitives(phys, eos, pr)
        sim.step(10)
        r = sim.fields()
        f = {key: v.cpu().numpy() for key, v in batch.fields(k).items()}
        ee, eu = e_err(f["e"], r["e"]), u_err(f["u"], r["u"], sim.tau)
        assert ee <= 1e-12 and eu <= 1e-12, (k, ee, eu)


def test_two_events_of_the_48_event_set_against_oracle(kt):
    """Two differently shaped events of the 48-event batch workload (event 7,
    64^3, and event 9, 96x96x64) advanced together for 10 steps, in FP64 and
    in the set's mixed-precision state, against the FP64 oracle run of each
    event: FP64 within 1e-9; mixed precision within 1e-6 (median cell) and
    1e-5 (dense cells, e > 1e-3 e_max), the bars of the 128^3 event."""
    shapes, _ = I.batch_shapes()
    assert tuple(shapes[[7, 9]]) == (0, 1)
    ws = I.workload_batch(only=(7, 9), mixed=False)
    refs = []
    for w in ws:
        sim = oracle.Simulation.from_primitives(oracle.Physics.from_config(w.grid, w.config), w.eos, w.prims)
        sim.step(10)
        refs.append((sim.fields(), sim.tau))
    for mixed in (False, True):
        evs = [(w.grid, dict(w.config, mixed=mixed), w.prims) for w in ws]
        batch = kt.Batch(evs, ws[0].eos)
        batch.tune()
        batch.step(10)
        for k, (r, tau) in enumerate(refs):
            f = {key: v.cpu().numpy() for key, v in batch.fields(k, ("e", "u")).items()}
            emax = r["e"].max()
            de = np.abs(f["e"] - r["e"]) / np.maximum(r["e"], 1e-6 * emax)
            du = np.max(np.abs(f["u"] - r["u"]) * np.array([1, 1, 1, tau])[:, None, None, None]
                        / r["u"][0:1], axis=0)
            dense = r["e"] > 1e-3 * emax
            print("batch event %d (%s), %s: e %.2e u %.2e, dense e %.2e, median e %.1e" % (
                (7, 9)[k], "x".join(map(str, ws[k].grid.shape[::-1])), "mixed" if mixed else "fp64",
                de.max(), du.max(), de[dense].max(), np.median(de)), flush=True)
            if mixed:
                assert np.median(de) <= 1e-6 and np.median(du) <= 1e-6
                assert de[dense].max() <= 1e-5 and du[dense].max() <= 1e-5
            else:
                assert de.max() <= 1e-9 and du.max() <= 1e-9
        batch.close()


def test_batch_with_poisoned_workspace(kt):
    """A batch workspace filled with 0xFF bytes (NaN in every floating-point
    view) gives the fields of a zero-filled one, bit for bit, after replays of
    the step graph: no batched kernel reads unwritten memory."""
    import ctypes as C
    import torch
    evs, eos = events(mixed=True)
    n = len(evs)
    params = (kt.KtParams * n)(*[kt.make_params(g, cfg, evs[0][2].tau0) for g, cfg, _ in evs])
    nbytes = int(kt.lib().kt_batch_workspace_bytes(params, n, C.byref(kt.EosHost(eos).c)))
    runs = []
    for fill in (0x00, 0xFF):
        b = kt.Batch(evs, eos, workspace=torch.full((nbytes,), fill, dtype=torch.uint8, device="cuda"))
        b.step(5)
        runs.append([b.fields(k) for k in range(n)])
        b.close()
    for k in range(n):
        assert same(runs[0][k], runs[1][k]), k
