"""Pins of the learned-start oracle (oracle/mlp.py) against facts that do not
come from the oracle itself: the normal distribution function, finite
differences of the forward pass, Adam's closed-form behaviour, exact states
whose features and targets are known, and the inversion's own convergence."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_1608_06577_amd import inputs as I

from tests.test_oracle_algebra import pack_pi, random_state


@pytest.fixture(scope="module")
def oracle_lib():
    oracle.build(force=False)
    return oracle.lib()


def test_parameter_count():
    assert M.N_PARAMS == 5188 == I.MLP_N_PARAMS
    assert I.mlp_init_params(3).shape == (5188,)


def test_gelu_pins():
    # Phi(1) and Phi(-1.5) from tables of the standard normal distribution
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(-1.5) - (-1.5 * 0.0668072012688581)) < 1e-15
    assert M.gelu(0.0) == 0.0
    # Phi(a) + Phi(-a) = 1  =>  gelu(a) - gelu(-a) = a
    a = np.linspace(-6, 6, 101)
    assert np.max(np.abs(M.gelu(a) - M.gelu(-a) - a)) < 1e-14
    # asymptotes
    assert abs(M.gelu(12.0) - 12.0) < 1e-15 and abs(M.gelu(-12.0)) < 1e-15
    # derivative against central differences
    h = 1e-5
    fd = (M.gelu(a + h) - M.gelu(a - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(a))) < 1e-9


def test_forward_special_cases():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, M.N_IN))
    theta = np.zeros(M.N_PARAMS)
    P = M.unpack(theta)
    # every parameter zero but the output bias: y = b3
    theta2 = theta.copy()
    M.unpack(theta2)["b3"][:] = [0.3, -1.0, 2.0, 0.5]
    y, _ = M.forward(theta2, x)
    assert np.array_equal(y, np.tile([0.3, -1.0, 2.0, 0.5], (7, 1)))
    # one path: x_f -> hidden 5 -> hidden 9 -> output 2, all scalars
    th = np.zeros(M.N_PARAMS)
    Q = M.unpack(th)
    Q["W1"][5, 3], Q["b1"][5] = 0.7, -0.2
    Q["W2"][9, 5], Q["b2"][9] = -1.3, 0.4
    Q["W3"][2, 9], Q["b3"][2] = 2.5, 0.1
    y, (a1, a2) = M.forward(th, x)
    Phi = lambda z: 0.5 * (1.0 + math.erf(z / math.sqrt(2.0)))
    for n in range(7):
        s1 = 0.7 * x[n, 3] - 0.2
        h1 = s1 * Phi(s1)
        s2 = -1.3 * h1 + 0.4
        h2 = s2 * Phi(s2)
        assert abs(y[n, 2] - (2.5 * h2 + 0.1)) < 1e-15
        assert y[n, 0] == 0.0 and y[n, 1] == 0.0 and y[n, 3] == 0.0
    del P


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = I.mlp_init_params(5).astype(np.float64)
    x = rng.standard_normal((9, M.N_IN))
    dy = rng.standard_normal((9, M.N_OUT))
    y, act = M.forward(theta, x)
    g = M.backward(theta, x, act, dy)
    f = lambda th: float(np.sum(dy * M.forward(th, x)[0]))
    idx = np.concatenate([rng.choice(M.N_PARAMS, 300, replace=False),
                          np.arange(704, 768), np.arange(5184, 5188)])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


@pytest.mark.parametrize("w", [None, (1.0, 0.1, 0.2, 0.05)])
def test_loss_gradient(w):
    rng = np.random.default_rng(2)
    y, t = rng.standard_normal((5, 4)), rng.standard_normal((5, 4))
    L, dy = M.loss_and_grad(y, t, w)
    wt = np.ones(4) if w is None else np.array(w)
    assert abs(L - sum(wt[o] * np.sum((y[:, o] - t[:, o]) ** 2) for o in range(4)) / 20) < 1e-15
    h = 1e-6
    for k in range(20):
        yp, ym = y.copy(), y.copy()
        yp.flat[k] += h
        ym.flat[k] -= h
        fd = (M.loss_and_grad(yp, t, w)[0] - M.loss_and_grad(ym, t, w)[0]) / (2 * h)
        assert abs(fd - dy.flat[k]) < 1e-9


def test_adam_closed_forms():
    rng = np.random.default_rng(3)
    th0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    # first step from zero moments: the bias-corrected moments are g and g^2
    th1, m, v = M.adam(th0, np.zeros(50), np.zeros(50), g, lr, b1, b2, eps, 1)
    assert np.max(np.abs(th1 - (th0 - lr * g / (np.abs(g) + eps)))) < 1e-15
    # a constant gradient keeps the corrected moments at g and g^2 for every t
    th = th1
    for t in range(2, 40):
        th_new, m, v = M.adam(th, m, v, g, lr, b1, b2, eps, t)
        assert np.max(np.abs((th - th_new) - lr * g / (np.abs(g) + eps))) < 1e-13
        th = th_new


def test_features_and_targets_of_known_states(oracle_lib):
    eos = I.eos_c1_table()
    tau = 0.8
    phys = oracle.Physics.from_config(I.Grid(1, 1, 1, 1, 1, 1), I.default_config(eta_s=0.2, zeta_coef=0.1))
    # fluid at rest without dissipation: x = (0, ..., 0, ln e / 10, c_s^2(e), p(e)/e), y = (1, 0, 0, 0)
    e = np.array([0.01, 1.0, 40.0, 300.0])
    q9 = np.zeros((4, 9))
    q9[:, 0] = e
    x = M.features(tau, False, q9, eos)
    p, cs2, _ = oracle.eos_eval(eos, e)
    assert np.all(x[:, :8] == 0.0)
    assert np.allclose(x[:, 8], np.log(e) / 10, rtol=0, atol=1e-15)
    assert np.array_equal(x[:, 9], cs2) and np.allclose(x[:, 10], p / e, rtol=1e-15)
    u = np.tile([1.0, 0.0, 0.0, 0.0], (4, 1))
    assert np.allclose(M.targets(tau, False, q9, e, u, 1e-9), np.tile([1.0, 0, 0, 0], (4, 1)), atol=1e-15)
    # moving viscous states: targets of the recovered state equal those of the primitives
    ev, uv, pi, Pi = random_state(tau, 200, u_scale=1.2)
    q = oracle.tmunu(phys, eos, tau, ev, uv, pack_pi(pi), Pi)
    q9 = q[:, [0, 1, 2, 3, 4, 5, 6, 7, 14]]
    er, ur, _, fl = oracle.recover(phys, eos, tau, q)
    assert np.all(fl == 0)
    t_rec = M.targets(tau, False, q9, er, ur, 1e-9)
    # conformal root of the same (E, M): for p = e/3, e = E - M^2/(E + e/3) is a
    # quadratic whose positive root is sqrt(4E^2 - 3M^2) - E
    E = q[:, 0] - q[:, 4]
    Ml = np.stack([q[:, 1] - q[:, 5], q[:, 2] - q[:, 6], q[:, 3] - q[:, 7]], 1)
    M2 = Ml[:, 0] ** 2 + Ml[:, 1] ** 2 + tau * tau * Ml[:, 2] ** 2
    ec = M.conformal_root(tau, False, q9, 1e-9)
    assert np.max(np.abs(ec - (E - M2 / (E + ec / 3.0))) / ec) < 1e-13
    t_true = np.stack([ev / ec, uv[:, 1] / uv[:, 0], uv[:, 2] / uv[:, 0], tau * uv[:, 3] / uv[:, 0]], 1)
    assert np.max(np.abs(t_rec - t_true)) < 1e-12
    # x_0 = T^{tau x}/T^{tau tau} with T^{tau mu} = (e + P) u^tau u^mu - P g^{tau mu} + pi^{tau mu}
    x = M.features(tau, False, q9, eos)
    P0, _, _ = oracle.eos_eval(eos, ev)
    w = (ev + P0 + Pi) * uv[:, 0]
    Ttt = w * uv[:, 0] - (P0 + Pi) + pi[:, 0, 0]
    assert np.max(np.abs(x[:, 0] - (w * uv[:, 1] + pi[:, 0, 1]) / Ttt)) < 1e-13
    assert np.max(np.abs(x[:, 2] - tau * (w * uv[:, 3] + pi[:, 0, 3]) / Ttt)) < 1e-13
    assert np.max(np.abs(x[:, 6] - tau * pi[:, 0, 3] / Ttt)) < 1e-13
    assert np.max(np.abs(x[:, 7] - Pi / Ttt)) < 1e-13


def test_recover_from_a_given_start(oracle_lib):
    eos = I.eos_c1_table()
    tau = 0.7
    phys = oracle.Physics.from_config(I.Grid(1, 1, 1, 1, 1, 1), I.default_config(eta_s=0.2, zeta_coef=0.1))
    ev, uv, pi, Pi = random_state(tau, 500, u_scale=1.5)
    q = oracle.tmunu(phys, eos, tau, ev, uv, pack_pi(pi), Pi)
    e0, u0, it0, fl0 = oracle.recover(phys, eos, tau, q)
    e1, u1, it1, fl1 = oracle.recover(phys, eos, tau, q, e_start=np.full(500, -1.0))
    assert np.array_equal(e0, e1) and np.array_equal(it0, it1)
    # started at the root, Newton stops after its first iteration
    e2, u2, it2, fl2 = oracle.recover(phys, eos, tau, q, e_start=ev)
    assert np.all(it2 == 1) and np.all(fl2 == 0)
    assert np.max(np.abs(e2 - ev) / ev) < 1e-13
    assert np.max(np.abs(u2 - uv) / uv[:, :1]) < 1e-12
    # a far start costs more iterations but reaches the same root
    e3, _, it3, _ = oracle.recover(phys, eos, tau, q, e_start=10.0 * ev)
    assert np.mean(it3) > np.mean(it2) and np.max(np.abs(e3 - ev) / ev) < 1e-13


def test_oracle_training_reduces_the_loss():
    """Adam on the oracle's own gradients fits a smooth 4-output map."""
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (128, M.N_IN))
    t = np.stack([np.sin(x[:, 0]) + 0.5, x[:, 1] * x[:, 2], np.cos(x[:, 8]), x[:, 9] ** 2], 1)
    theta = I.mlp_init_params(1).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = None
    for step in range(1, 301):
        y, act = M.forward(theta, x)
        L, dy = M.loss_and_grad(y, t)
        L0 = L if L0 is None else L0
        theta, m, v = M.adam(theta, m, v, M.backward(theta, x, act, dy), 3e-3, 0.9, 0.999, 1e-8, step)
    assert L < 0.05 * L0
