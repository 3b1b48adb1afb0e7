"""Pins of the oracle's temperature-dependent bulk viscosity (Sec. 2.2,
Eq. zetas) and of its use in the relaxation rate of Pi."""
import numpy as np

import oracle
from paper_1608_06577_amd import inputs as I


def test_zeta_over_s_shape():
    f = oracle.zeta_over_s_paper
    # the three branches meet (the fit is continuous to its printed digits)
    for x0 in (0.995, 1.05):
        lo, hi = float(f(x0 - 1e-12)), float(f(x0 + 1e-12))
        assert abs(lo - hi) < 0.02 * hi, (x0, lo, hi)
    # asymptotic values of the QGP and hadron-gas tails
    assert abs(float(f(20.0)) - 0.001) < 1e-12
    assert abs(float(f(0.2)) - 0.03) < 1e-12
    # the peak sits at T_c, and three times the curve peaks at 1 (the text's
    # normalisation 3 "has a peak value of 1")
    x = np.linspace(0.9, 1.2, 30001)
    y = f(x)
    assert abs(x[np.argmax(y)] - 1.0) < 2e-3
    assert 0.98 < 3.0 * y.max() <= 1.0
    # monotone on both sides of the peak
    assert np.all(np.diff(y[x > 1.001]) < 0) and np.all(np.diff(y[x < 0.999]) > 0)


def test_bulk_relaxation_rate_uses_the_model():
    """A uniform fluid at rest in a periodic Cartesian box: no gradients, so
    dPi/dt = -Pi / tau_Pi, with zeta / tau_Pi = 15 (1/3 - c_s^2)^2 (e + P) and
    zeta = (zeta/s) (e + P) / T."""
    g = I.Grid(4, 3, 2, 0.3, 0.3, 0.3)
    eos = I.eos_lattice_table(n=1024)
    prims = I.random_smooth_fields(g, 1.0, seed=5, cartesian=True, e_mean=2.0)
    e0, Pi0 = 2.5, 0.04
    prims.e[...] = e0
    prims.u[...] = 0.0
    prims.u[0] = 1.0
    prims.pi[...] = 0.0
    prims.Pi[...] = Pi0
    p, cs2, T = oracle.eos_eval(eos, np.array([e0]))
    d = 1.0 / 3.0 - cs2[0]
    tc = 0.2 / I.HBARC
    for model, norm in ((0, 0.1), (1, 1.0), (1, 2.5)):
        cfg = I.default_config(cartesian=True, periodic=(True, True, True), zeta_coef=norm,
                               zeta_model=model, zeta_tc=tc, eta_s=0.0, regulate=False)
        phys = oracle.Physics.from_config(g, cfg)
        sim = oracle.Simulation.from_primitives(phys, eos, prims)
        J = sim.rhs()
        zs = norm * d if model == 0 else norm * float(oracle.zeta_over_s_paper(T[0] / tc))
        rate = 15.0 * d * d * T[0] / zs
        dPi = np.asarray(J).reshape(-1, 15)[:, 14] if np.ndim(J) == 2 else np.asarray(J)[14::15]
        assert np.allclose(dPi, -Pi0 * rate, rtol=1e-12, atol=0), (model, norm, dPi[:3], -Pi0 * rate)


def test_inverse_reynolds_numbers_closed_forms():
    """Sec. 7: a Navier-Stokes Bjorken state has pi^{xx} = pi^{yy} = pi_s/2,
    tau^2 pi^{eta eta} = -pi_s, so sqrt(pi:pi) = sqrt(3/2) pi_s; and pi:pi is
    a Lorentz scalar (unchanged by a boost of the tensor)."""
    eos = I.eos_c1_table(n=512)
    tau, e, pis, Pi = 1.7, np.array([3.0, 11.0]), np.array([0.4, 1.3]), np.array([-0.05, 0.2])
    pi = np.zeros((10, 2))
    pi[4] = pi[7] = 0.5 * pis
    pi[9] = -pis / tau ** 2
    T, rpi, rPi = oracle.validity_maps(eos, tau, False, e, pi, Pi)
    p, _, T_ref = oracle.eos_eval(eos, e)
    assert np.allclose(rpi, np.sqrt(1.5) * pis / p, rtol=1e-14, atol=0)
    assert np.allclose(rPi, np.abs(Pi) / p, rtol=1e-15, atol=0) and np.array_equal(T, T_ref)
    # boost invariance (Cartesian metric)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(3, 3))
    full = np.zeros((4, 4))
    full[1:, 1:] = a + a.T          # rest-frame tensor: pi:pi = sum of squares > 0
    y = 0.7
    L = np.eye(4)
    L[0, 0] = L[1, 1] = np.cosh(y)
    L[0, 1] = L[1, 0] = np.sinh(y)
    boosted = L @ full @ L.T
    pack = lambda M: np.array([M[m, n] for (m, n) in ((0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2),
                                                      (1, 3), (2, 2), (2, 3), (3, 3))])[:, None]
    g = np.diag([1.0, -1.0, -1.0, -1.0])
    pp = np.trace(g @ full @ g @ full.T)
    r0 = oracle.validity_maps(eos, 1.0, True, np.array([5.0]), pack(full), np.array([0.0]))[1]
    r1 = oracle.validity_maps(eos, 1.0, True, np.array([5.0]), pack(boosted), np.array([0.0]))[1]
    p5 = oracle.eos_eval(eos, np.array([5.0]))[0][0]
    assert pp > 0 and abs(r0[0] - np.sqrt(pp) / p5) <= 1e-12 * r0[0]
    assert not np.allclose(pack(boosted)[:4], 0.0)      # the boost mixes in tau components
    assert abs(r0[0] - r1[0]) <= 1e-11 * r0[0]
