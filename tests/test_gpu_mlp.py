"""Parity of the learned-start kernels (through the C ABI) with the FP64
oracle (oracle/mlp.py), and what the trained network gains.

FP32 kernels against FP64 references: tolerances follow from FP32 rounding
(unit roundoff 6e-8) accumulated over at most 64-term dot products and the
sums over samples."""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_1608_06577_amd import inputs as I

from tests.test_oracle_algebra import pack_pi, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kt():
    import torch
    assert torch.cuda.is_available()
    from paper_1608_06577_amd import kt as K
    K.lib()
    return K


def tiny_solver(kt, eos=None, cartesian=False):
    g = I.Grid(4, 4, 4, 0.2, 0.2, 0.2)
    cfg = I.default_config(eta_s=0.2, zeta_coef=0.1, cartesian=cartesian)
    prims = I.random_smooth_fields(g, 0.8, seed=2, e_mean=3.0, cartesian=cartesian)
    return kt.Solver(g, cfg, eos or I.eos_c1_table(), prims), cfg


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def states(n, tau):
    """Random physical states (the shared generator of the oracle tests)."""
    return random_state(tau, n, u_scale=1.3)


@pytest.mark.parametrize("cartesian", [False, True])
def test_features_and_targets_match_oracle(kt, cartesian):
    eos = I.eos_c1_table()
    gpu, cfg = tiny_solver(kt, eos, cartesian)
    tau = 0.9
    phys = oracle.Physics.from_config(I.Grid(1, 1, 1, 1, 1, 1), cfg)
    ev, uv, pi, Pi = states(3000, 1.0 if cartesian else tau)
    q = oracle.tmunu(phys, eos, tau, ev, uv, pack_pi(pi), Pi)
    q9 = q[:, [0, 1, 2, 3, 4, 5, 6, 7, 14]]
    e_r, u_r, _, fl = oracle.recover(phys, eos, tau, q)
    x_o = M.features(tau, cartesian, q9, eos)
    t_o = M.targets(tau, cartesian, q9, e_r, u_r, cfg["e_floor"])
    ins = [dev(q9[:, k]) for k in range(9)]
    x, t = gpu.mlp_features(ins, tau, dev(e_r), dev(u_r.T))
    x, t = x.cpu().numpy().T, t.cpu().numpy().T
    assert np.max(np.abs(x - x_o) / np.maximum(1.0, np.abs(x_o))) < 3e-7
    assert np.max(np.abs(t - t_o) / np.maximum(1.0, np.abs(t_o))) < 3e-7


def test_forward_matches_oracle(kt):
    gpu, _ = tiny_solver(kt)
    theta = I.mlp_init_params(7)
    gpu.mlp_set(dev(theta))
    rng = np.random.default_rng(3)
    n = 2500
    x = rng.uniform(-2, 2, (n, 11)).astype(np.float32)
    y_o, (a1_o, a2_o) = M.forward(theta.astype(np.float64), x.astype(np.float64))
    y, act = gpu.mlp_fwd(dev(x.T), keep_act=True)
    y, act = y.cpu().numpy().T, act.cpu().numpy().T
    assert np.max(np.abs(act[:, :64] - a1_o) / (1 + np.abs(a1_o))) < 2e-6
    assert np.max(np.abs(act[:, 64:] - a2_o) / (1 + np.abs(a2_o))) < 2e-5
    assert np.max(np.abs(y - y_o) / (1 + np.abs(y_o))) < 2e-5
    # the parameters come back unchanged
    assert np.array_equal(gpu.mlp_get().cpu().numpy(), theta)


def test_matrix_core_start_matches_oracle(kt):
    """y_0 from the recoveries' matrix-core inference (kt_mlp_y0) against the
    oracle network.  The inference rounds the features, W1, W2 and the first
    hidden layer's activations to FP16 (unit roundoff 2^-11): against the
    oracle evaluated with the same roundings the remaining differences are FP32
    accumulation, the erf approximation (< 1.5e-7) and the occasional FP16
    rounding of a first-layer activation that falls the other way (one unit
    changes y_0 by |W3 W2| 2^-11 ~ 1e-4), bar 1e-3; against the exact FP64
    network the FP16 roundings themselves, bar 2e-2 (both absolute, y_0 ~ 1)."""
    gpu, _ = tiny_solver(kt)
    theta = I.mlp_init_params(7)
    gpu.mlp_set(dev(theta))
    rng = np.random.default_rng(4)
    n = 3000
    x = rng.uniform(-1.5, 1.5, (n, 11)).astype(np.float32)
    y0 = gpu.mlp_y0(dev(x.T)).cpu().numpy().astype(np.float64)
    y_exact = M.forward(theta.astype(np.float64), x.astype(np.float64))[0][:, 0]
    P = M.unpack(theta.astype(np.float64))
    h16 = lambda a: np.asarray(a, np.float16).astype(np.float64)
    a1 = h16(x) @ h16(P["W1"]).T + P["b1"]
    a2 = h16(M.gelu(a1)) @ h16(P["W2"]).T + P["b2"]
    y_half = M.gelu(a2) @ P["W3"][0] + P["b3"][0]
    d_half, d_exact = np.abs(y0 - y_half).max(), np.abs(y0 - y_exact).max()
    print("matrix-core y_0: max |d| %.2e against the FP16-rounded oracle, %.2e against the exact "
          "network (|y_0| up to %.2f)" % (d_half, d_exact, np.abs(y_exact).max()), flush=True)
    assert d_half < 1e-3 and d_exact < 2e-2
    # lanes past n (a partial wave) and n = 1
    y1 = gpu.mlp_y0(dev(x[:1].T)).cpu().numpy()
    assert abs(float(y1[0]) - y0[0]) == 0.0


@pytest.mark.parametrize("n", [1, 37, 5000])
def test_backward_matches_oracle(kt, n):
    """Sizes: one sample, a ragged chunk, many blocks with a ragged tail."""
    gpu, _ = tiny_solver(kt)
    theta = I.mlp_init_params(11)
    gpu.mlp_set(dev(theta))
    rng = np.random.default_rng(n)
    x = rng.uniform(-2, 2, (n, 11)).astype(np.float32)
    dy = rng.standard_normal((n, 4)).astype(np.float32)
    th = theta.astype(np.float64)
    y_o, act_o = M.forward(th, x.astype(np.float64))
    g_o = M.backward(th, x.astype(np.float64), act_o, dy.astype(np.float64))
    y, act = gpu.mlp_fwd(dev(x.T), keep_act=True)
    g = gpu.mlp_bwd(dev(x.T), act, dev(dy.T)).cpu().numpy()
    for name, shp in M.SHAPES:
        a, b = M.unpack(g.astype(np.float64))[name], M.unpack(g_o)[name]
        scale = max(np.abs(b).max(), 1e-30)
        assert np.max(np.abs(a - b)) <= 1e-4 * scale, (name, np.max(np.abs(a - b)) / scale)


def test_loss_and_adam_match_oracle(kt):
    gpu, _ = tiny_solver(kt)
    theta = I.mlp_init_params(2)
    gpu.mlp_set(dev(theta))
    rng = np.random.default_rng(9)
    n = 3000
    y = rng.standard_normal((n, 4)).astype(np.float32)
    t = rng.standard_normal((n, 4)).astype(np.float32)
    for w in (None, (1.0, 0.125, 0.25, 0.0625)):   # weights exact in FP32
        L_o, dy_o = M.loss_and_grad(y.astype(np.float64), t.astype(np.float64), w)
        L, dy = gpu.mlp_loss(dev(y.T), dev(t.T), w)
        assert abs(L.item() - L_o) < 1e-12 * L_o
        assert np.max(np.abs(dy.cpu().numpy().T - dy_o)) < 1e-7 * np.abs(dy_o).max()
    th, m, v = theta.astype(np.float64), np.zeros(5188), np.zeros(5188)
    for step in range(1, 6):
        g = rng.standard_normal(5188).astype(np.float32)
        gpu.mlp_adam(dev(g), step, lr=1e-3)
        th, m, v = M.adam(th, m, v, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, step)
    got = gpu.mlp_get().cpu().numpy()
    assert np.max(np.abs(got - th)) < 2e-6


def test_learned_start_against_conformal_start(kt):
    """Train on a hot-spot event's own states, then invert held-out states of
    a different event.  The inversion results equal the oracle's whatever the
    start, and the network's start is closer to the root than the conformal
    closed form (median over the states): that is what the network gains.
    It gains no Newton iteration: convergence is quadratic, so at the 1e-12
    tolerance a start saves an iteration only below ~1e-6 relative error, and
    both starts (~1e-3) take about the same number of iterations; the test
    reports them without a bar.  The full step with the learned start then
    matches the FP64 oracle to the 1e-9 bar, like the plain step."""
    import torch
    w = I.workload_hotspot(nx=40, ny=40, neta=16, dx=0.4, deta=0.5, n_hot=40, seed=5)
    gpu = kt.Solver(w.grid, w.config, w.eos, w.prims)
    gpu.mlp_set(dev(I.mlp_init_params(0)))
    from paper_1608_06577_amd import learned
    X, T = learned.collect_pairs(gpu, w.config["e_floor"], n_snap=6, steps_between=10)
    losses = learned.train(gpu, X, T, steps=3000)
    print("training loss:", ["%.2e" % l for l in losses], flush=True)
    assert losses[-1] < 0.01 * losses[0]
    # held-out states: another event, later time
    w2 = I.workload_hotspot(nx=40, ny=40, neta=16, dx=0.4, deta=0.5, n_hot=60, seed=9)
    other = kt.Solver(w2.grid, w2.config, w2.eos, w2.prims)
    other.step(25)
    f = other.fields(("q",))
    tau = other.observables()["tau"]
    q = f["q"].reshape(15, -1)
    keep = q[0] > 10 * w.config["e_floor"]
    ins = [q[k][keep].contiguous() for k in (0, 1, 2, 3, 4, 5, 6, 7, 14)]
    gpu.set_inv_start(kt.KT_START_CONFORMAL)
    e_c, u_c, it_c, fl_c = gpu.recover(ins, tau)
    gpu.set_inv_start(kt.KT_START_LEARNED)
    e_l, u_l, it_l, fl_l = gpu.recover(ins, tau)
    phys = oracle.Physics.from_config(w.grid, w.config)
    qa = q[:, keep].T.cpu().numpy()
    e_o, u_o, it_o, fl_o = oracle.recover(phys, w.eos, tau, qa)
    e_l, u_l = e_l.cpu().numpy(), u_l.cpu().numpy().T
    assert np.array_equal(fl_l.cpu().numpy() & 1, fl_o & 1)
    assert np.max(np.abs(e_l - e_o) / e_o) < 1e-13
    assert np.max(np.abs(u_l - u_o) / u_o[:, :1]) < 1e-12
    # start errors: the network's y_0 e_c against the conformal root e_c
    q9 = qa[:, [0, 1, 2, 3, 4, 5, 6, 7, 14]]
    ec = M.conformal_root(tau, False, q9, w.config["e_floor"])
    y0 = gpu.mlp_fwd(gpu.mlp_features(ins, tau))[0].double().cpu().numpy()
    err_c, err_l = np.abs(ec - e_o) / e_o, np.abs(y0 * ec - e_o) / e_o
    mc, ml = it_c.double().mean().item(), it_l.double().mean().item()
    print("held-out states %d: median start error conformal %.2e learned %.2e; "
          "Newton iterations per state conformal %.3f learned %.3f"
          % (len(e_o), np.median(err_c), np.median(err_l), mc, ml), flush=True)
    assert np.median(err_l) < np.median(err_c)
    # the full step with the learned start: equal to the step with the warm
    # start to rounding, and to the FP64 oracle within the 1e-9 bar
    gw = kt.Solver(w2.grid, w2.config, w2.eos, w2.prims)
    gl = kt.Solver(w2.grid, w2.config, w2.eos, w2.prims)
    gl.mlp_set(gpu.mlp_get())
    gl.set_inv_start(kt.KT_START_LEARNED)
    gw.set_inv_start(kt.KT_START_WARM)
    gw.step(20)
    gl.step(20)
    a, b = gw.fields(("e",))["e"], gl.fields(("e",))["e"]
    assert (torch.abs(a - b) / a).max().item() < 1e-12
    sim = oracle.Simulation.from_primitives(oracle.Physics.from_config(w2.grid, w2.config), w2.eos, w2.prims)
    sim.step(20)
    r = sim.fields()
    fl = {k: v.cpu().numpy() for k, v in gl.fields(("e", "u")).items()}
    emax = r["e"].max()
    de = np.max(np.abs(fl["e"] - r["e"]) / np.maximum(r["e"], 1e-6 * emax))
    du = np.max(np.abs(fl["u"] - r["u"]) * np.array([1, 1, 1, sim.tau])[:, None, None, None] / r["u"][0:1])
    print("learned-start step vs oracle, 20 steps: e %.2e u %.2e" % (de, du), flush=True)
    assert de <= 1e-9 and du <= 1e-9
    ow, ol = gw.observables(), gl.observables()
    print("kt_step cell iterations: warm %.3f, learned %.3f" % (
        ow["newton_iters_cells"] / ow["n_recover_cells"], ol["newton_iters_cells"] / ol["n_recover_cells"]),
        flush=True)


def test_learned_start_needs_parameters(kt):
    gpu, _ = tiny_solver(kt)
    with pytest.raises(kt.KtError) as ei:
        gpu.set_inv_start(kt.KT_START_LEARNED)
    assert ei.value.status == kt.KT_E_STATE
    with pytest.raises(kt.KtError):
        gpu.set_inv_start(7)
