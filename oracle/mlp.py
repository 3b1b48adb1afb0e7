"""FP64 oracle of the learned start of the cell inversion.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this module.  It shares no code with the HIP path.

The cell inversion of Sec. 2.4 / Sec. 3.2 (e from T^{tau mu}, pi^{tau mu},
Pi by Newton's method on f(e) = e - E + M^2/(E + p(e) + Pi)) needs a
starting value.  Here a small network proposes it:

  features x (11): T^{tau x}/T^{tau tau}, T^{tau y}/T^{tau tau},
      sqrt(g33) T^{tau eta}/T^{tau tau}, pi^{tau tau}/T^{tau tau},
      pi^{tau x}/T^{tau tau}, pi^{tau y}/T^{tau tau},
      sqrt(g33) pi^{tau eta}/T^{tau tau}, Pi/T^{tau tau},
      ln(T^{tau tau})/10, c_s^2(T^{tau tau}), p(T^{tau tau})/T^{tau tau}
      (g33 = tau^2 in Milne coordinates, 1 in Cartesian ones; c_s^2 and p of
      the equation of state evaluated at e = T^{tau tau});
  targets y (4): e/e_c and the velocity v^x = u^x/u^tau, v^y = u^y/u^tau,
      sqrt(g33) u^eta/u^tau, where e_c = sqrt(4E^2 - 3M^2) - E is the root for
      the conformal EOS without bulk (E = T^{tau tau} - pi^{tau tau}, M^2 =
      (T^{tau x} - pi^{tau x})^2 + (T^{tau y} - pi^{tau y})^2
      + g33 (T^{tau eta} - pi^{tau eta})^2), floored at e_floor;
  network: 11 -> 64 -> 64 -> 4, GELU(a) = a Phi(a) = a (1 + erf(a/sqrt 2))/2
      after the two hidden layers, linear output;
  start: e_0 = y_0 e_c, then the usual Newton polish.

Parameters are one flat vector of 5188 numbers: W1 (64 x 11, row major), b1
(64), W2 (64 x 64), b2 (64), W3 (4 x 64), b3 (4); a layer computes
a = W h + b.  The loss is the mean over samples and outputs of
w_o (y_o - t_o)^2 with per-output weights w (default 1); training uses Adam
(Kingma & Ba, arXiv:1412.6980, Algorithm 1).
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H, N_OUT = 11, 64, 4
SHAPES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 5188
LN_SCALE = 0.1                                       # x_8 = ln(T^{tau tau}) * LN_SCALE


def unpack(theta):
    """Views of the flat parameter vector, in the order of SHAPES."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[off:off + n].reshape(shp)
        off += n
    return out


def _erf(a):
    return np.vectorize(math.erf, otypes=[np.float64])(a)


def gelu(a):
    """a Phi(a), Phi the standard normal distribution function."""
    a = np.asarray(a, dtype=np.float64)
    return 0.5 * a * (1.0 + _erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    """d/da [a Phi(a)] = Phi(a) + a phi(a)."""
    a = np.asarray(a, dtype=np.float64)
    return 0.5 * (1.0 + _erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def forward(theta, x):
    """x (n, 11) -> y (n, 4) and the pre-activations (a1, a2), each (n, 64)."""
    P = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ P["W1"].T + P["b1"]
    a2 = gelu(a1) @ P["W2"].T + P["b2"]
    y = gelu(a2) @ P["W3"].T + P["b3"]
    return y, (a1, a2)


def backward(theta, x, act, dy):
    """Gradient (5188) of sum_samples <dy, y> with respect to the parameters,
    by the chain rule through the three layers."""
    P = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1, a2 = act
    h1, h2 = gelu(a1), gelu(a2)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    d2 = (dy @ P["W3"]) * gelu_grad(a2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * gelu_grad(a1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def loss_and_grad(y, t, w=None):
    """Mean over samples and outputs of w_o (y_o - t_o)^2, y and t (n, 4), and
    its gradient in y."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    wt = np.ones(N_OUT) if w is None else np.asarray(w, dtype=np.float64)
    n = d.size
    return float(np.sum(wt * d * d) / n), 2.0 * wt * d / n


def adam(theta, m, v, g, lr, b1, b2, eps, t):
    """One Adam step (t >= 1): returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(tau, cartesian, q9, eos):
    """q9 (n, 9): T^{tau mu}, pi^{tau mu}, Pi per cell -> x (n, 11).  eos is the
    oracle's equation of state (oracle.eos_eval)."""
    from . import eos_eval
    q9 = np.asarray(q9, dtype=np.float64)
    sg = 1.0 if cartesian else float(tau)
    T0 = q9[:, 0]
    p, cs2, _ = eos_eval(eos, T0)
    x = np.empty((q9.shape[0], N_IN))
    x[:, 0] = q9[:, 1] / T0
    x[:, 1] = q9[:, 2] / T0
    x[:, 2] = sg * q9[:, 3] / T0
    x[:, 3] = q9[:, 4] / T0
    x[:, 4] = q9[:, 5] / T0
    x[:, 5] = q9[:, 6] / T0
    x[:, 6] = sg * q9[:, 7] / T0
    x[:, 7] = q9[:, 8] / T0
    x[:, 8] = np.log(T0) * LN_SCALE
    x[:, 9] = cs2
    x[:, 10] = p / T0
    return x


def conformal_root(tau, cartesian, q9, e_floor):
    """e_c = sqrt(4E^2 - 3M^2) - E, floored at e_floor (M^2 above 4E^2/3 gives e_floor)."""
    q9 = np.asarray(q9, dtype=np.float64)
    g33 = 1.0 if cartesian else float(tau) ** 2
    E = q9[:, 0] - q9[:, 4]
    M2 = (q9[:, 1] - q9[:, 5]) ** 2 + (q9[:, 2] - q9[:, 6]) ** 2 + g33 * (q9[:, 3] - q9[:, 7]) ** 2
    return np.maximum(np.sqrt(np.maximum(4.0 * E * E - 3.0 * M2, 0.0)) - E, e_floor)


def targets(tau, cartesian, q9, e, u, e_floor):
    """Training targets from the recovered (e, u): (n, 4)."""
    q9 = np.asarray(q9, dtype=np.float64)
    sg = 1.0 if cartesian else float(tau)
    u = np.asarray(u, dtype=np.float64)
    ec = conformal_root(tau, cartesian, q9, e_floor)
    return np.stack([np.asarray(e) / ec, u[:, 1] / u[:, 0], u[:, 2] / u[:, 0],
                     sg * u[:, 3] / u[:, 0]], axis=1)
