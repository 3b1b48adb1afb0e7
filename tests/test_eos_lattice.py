"""Pins of the lattice-QCD EOS table generator (Sec. 2, equation of state for
nuclear collisions): thermodynamic identities checked by finite differences of
the table, an independent quadrature of the pressure integral, and the limits
the text states (pressure towards the Stefan-Boltzmann value, c_s^2 towards
1/3 from below, with a dip near the crossover)."""
import math

import numpy as np
import pytest

from paper_1608_06577_amd import inputs as I


@pytest.fixture(scope="module")
def lattice():
    return I.eos_lattice_table()


def test_thermodynamic_identities(lattice):
    eos = lattice
    e, p, T = eos.e_nodes(), eos.p, eos.T
    s = (e + p) / T
    # s = dp/dT and c_s^2 = dp/de, by central differences on the table's nodes
    # (second-order differences on a ln e step of 0.0056)
    dpdT = np.gradient(p, T)[1:-1]
    assert np.max(np.abs(dpdT - s[1:-1]) / s[1:-1]) < 2e-5
    dpde = np.gradient(p, e)[1:-1]
    assert np.max(np.abs(dpde - eos.cs2[1:-1]) / eos.cs2[1:-1]) < 1e-5
    assert np.all(np.diff(T) > 0) and np.all(np.diff(p) > 0)


def test_pressure_integral_by_quadrature(lattice):
    from scipy.integrate import quad
    eos = lattice
    for i in (0, 700, 1800, 2600, 3500, eos.n - 1):
        Tg = eos.T[i] * I.HBARC
        P = quad(lambda x: float(I.wb_trace_anomaly(math.exp(x))), math.log(0.002), math.log(Tg),
                 limit=400, epsabs=0.0, epsrel=1e-12)[0]
        assert abs(eos.p[i] / eos.T[i] ** 4 - P) <= 1e-9 * P, i
        # e = 3p + I at the node's temperature
        phi = float(I.wb_trace_anomaly(Tg))
        assert abs(eos.e_nodes()[i] / eos.T[i] ** 4 - (3.0 * P + phi)) <= 1e-9 * (3.0 * P + phi), i


def test_limits_stated_in_the_text(lattice):
    eos = lattice
    e, T = eos.e_nodes(), eos.T
    Tg = T * I.HBARC
    p_sb = I.A_SB_QCD / 3.0
    pT4 = eos.p / T ** 4
    # the pressure rises towards the Stefan-Boltzmann value and stays below it
    top = Tg > 0.3
    assert np.all(np.diff(pT4[top]) > 0) and pT4[-1] < p_sb and pT4[-1] > 0.8 * p_sb
    assert abs(A := I.A_SB_QCD - 47.5 * math.pi ** 2 / 30.0) < 1e-12, A
    # c_s^2 < 1/3, approaching it at high T; a minimum near the crossover
    assert np.all(eos.cs2 < 1.0 / 3.0) and eos.cs2[-1] > 0.32
    hot = Tg > 0.08
    i = np.argmin(np.where(hot, eos.cs2, np.inf))
    assert 0.12 < Tg[i] < 0.17 and 0.10 < eos.cs2[i] < 0.16
    # far above the table the integral converges (the alpha term): P(inf) within the SB value
    from scipy.integrate import quad
    Pinf = quad(lambda x: float(I.wb_trace_anomaly(math.exp(x))), math.log(0.002), math.log(2000.0),
                limit=400)[0]
    assert 0.85 * p_sb < Pinf < p_sb


def test_printed_exponent_sign_caps_the_pressure_lower():
    """The reading recorded for the fit's exponential factor: with the sign as
    printed the pressure saturates near 0.63 of the Stefan-Boltzmann value."""
    from scipy.integrate import quad
    p_sb = I.A_SB_QCD / 3.0
    P = {sg: quad(lambda x: float(I.wb_trace_anomaly(math.exp(x), sg)), math.log(0.002), math.log(2000.0),
                  limit=400)[0] for sg in (1.0, -1.0)}
    assert P[1.0] < 0.65 * p_sb < 0.85 * p_sb < P[-1.0]
