"""Pins for the oracle's FP64 hazards.

Proposition 1 (stable log-normal hazard) is checked against the direct
density/survival ratio f/S from scipy.stats and against 50-digit mpmath;
erfcx against scipy.special.erfcx and mpmath; the Weibull and Erlang hazards
against scipy.stats pdf/sf; special cases that reduce to the exponential law;
and the limits tau -> 0 and tau -> infinity.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import special, stats

mpmath.mp.dps = 50


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_erfcx_vs_scipy_dense(orc):
    z = np.concatenate([np.linspace(-26.5, 30.0, 200_001), np.geomspace(30.0, 1e8, 2001)])
    ours = orc.erfcx(z)
    ref = special.erfcx(z)
    assert rel(ours, ref).max() < 2e-13


@pytest.mark.parametrize("z", [-26.0, -12.5, -4.81, -3.26, -1.0, -1e-3, 0.0, 1e-8, 0.5, 3.5,
                               9.0, 24.999, 25.0, 40.0, 1e3, 1e6])
def test_erfcx_vs_mpmath(orc, z):
    zm = mpmath.mpf(z)
    ref = mpmath.exp(zm * zm) * mpmath.erfc(zm)
    assert abs(orc.erfcx(z)[0] - float(ref)) <= 2e-14 * float(ref)


def test_erfcx_beyond_range(orc):
    assert np.isinf(orc.erfcx(-27.0)[0])


def lognormal_mp(tau, mu, sigma):
    t = mpmath.mpf(tau)
    m = mpmath.mpf(mu)
    s = mpmath.mpf(sigma)
    zz = (mpmath.log(t) - m) / s
    f = mpmath.exp(-zz * zz / 2) / (t * s * mpmath.sqrt(2 * mpmath.pi))
    S = mpmath.erfc(zz / mpmath.sqrt(2)) / 2
    return f / S


@pytest.mark.parametrize("mu,sigma", [(math.log(3), 0.5), (math.log(5), 0.6),
                                      (math.log(4), 0.668), (math.log(2), 0.3),
                                      (math.log(6), 0.8)])
def test_lognormal_vs_mpmath(orc, mu, sigma):
    taus = np.concatenate([np.geomspace(1e-3, 1e4, 300), np.arange(1, 600) * 0.1])
    ours = orc.hazard(("lognormal", mu, sigma), taus)
    ref = np.array([float(lognormal_mp(t, mu, sigma)) for t in taus])
    assert rel(ours, ref).max() < 5e-13


def test_lognormal_vs_scipy_f_over_s(orc):
    mu, sigma = math.log(3.0), 0.5
    taus = np.geomspace(0.05, 200.0, 5000)
    d = stats.lognorm(s=sigma, scale=math.exp(mu))
    ref = d.pdf(taus) / d.sf(taus)
    assert rel(orc.hazard(("lognormal", mu, sigma), taus), ref).max() < 1e-11


def test_prop1_worked_point(orc):
    # tau = 2, mu = ln 3, sigma = 0.5: erfcx form equals f/S (Proposition 1)
    d = stats.lognorm(s=0.5, scale=3.0)
    assert rel(orc.hazard(("lognormal", math.log(3), 0.5), [2.0])[0], d.pdf(2.0) / d.sf(2.0)) < 1e-14


def test_lognormal_limits(orc):
    mu, sigma = math.log(3.0), 0.5
    h = orc.hazard(("lognormal", mu, sigma), [0.0, 1e-6, 1e-3])
    assert h[0] == 0.0 and h[1] < 1e-100 and h[2] < 1e-20
    # tau -> infinity: h ~ (ln tau - mu) / (sigma^2 tau)
    for tau in [1e10, 1e30, 1e100]:
        ratio = orc.hazard(("lognormal", mu, sigma), [tau])[0] * sigma**2 * tau / (math.log(tau) - mu)
        assert abs(ratio - 1.0) < sigma**2 / (math.log(tau) - mu) ** 2 * 1.5


@pytest.mark.parametrize("shape,scale", [(2.0, 6.0), (1.5, 3.0), (3.0, 8.0), (2.37, 4.1)])
def test_weibull_vs_scipy(orc, shape, scale):
    taus = np.concatenate([np.geomspace(1e-4, 60.0, 3000), [0.0]])
    d = stats.weibull_min(c=shape, scale=scale)
    ref = d.pdf(taus) / d.sf(taus)
    ref[-1] = 0.0
    assert rel(orc.hazard(("weibull", shape, scale), taus), ref).max() < 1e-12


@pytest.mark.parametrize("k,rate", [(3, 1.0), (2, 0.5), (5, 1.25), (4, 2.0 / 3.0)])
def test_erlang_vs_scipy(orc, k, rate):
    taus = np.concatenate([np.geomspace(1e-4, 40.0, 3000), [0.0]])
    d = stats.gamma(a=k, scale=1.0 / rate)
    ref = d.pdf(taus) / d.sf(taus)
    ref[-1] = 0.0
    assert rel(orc.hazard(("erlang", k, rate), taus), ref).max() < 1e-12


def test_exponential_special_cases(orc):
    taus = np.linspace(0.0, 30.0, 301)
    np.testing.assert_allclose(orc.hazard(("weibull", 1.0, 4.0), taus), 0.25, rtol=0, atol=0)
    np.testing.assert_allclose(orc.hazard(("erlang", 1, 0.7), taus), 0.7, rtol=1e-15)
    np.testing.assert_allclose(orc.hazard(("exp", 0.3), taus), 0.3, rtol=0, atol=0)


def test_erlang_tends_to_rate(orc):
    h = orc.hazard(("erlang", 3, 1.0), [1e3, 1e6])
    assert abs(h[0] - 1.0) < 3e-3 and abs(h[1] - 1.0) < 3e-6


def test_erlang_k3_closed_form(orc):
    # k = 3, rate 1: h = (x^2/2) / (1 + x + x^2/2)
    x = np.linspace(0.0, 20.0, 201)
    np.testing.assert_allclose(orc.hazard(("erlang", 3, 1.0), x), (x**2 / 2) / (1 + x + x**2 / 2),
                               rtol=1e-14, atol=0)
