"""Pins of the oracle's adaptive step size (Section "Bernoulli tau-leaping",
adaptive step selection; the tau update of Algorithm 3): the rule itself,
the reduction to the fixed-step scheme, and an exact law for constant rates
under a varying step."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def test_next_dt_rule():
    # min(dt_max, eps / (lam_max + delta))
    assert oracle.next_dt(0.0, 0.03, 0.1) == 0.1          # no positive rate: the cap
    assert oracle.next_dt(1.0, 0.03, 0.1) == pytest.approx(0.03, rel=1e-15)
    assert oracle.next_dt(0.2, 0.03, 0.1) == 0.1          # eps/lam = 0.15 > cap
    assert oracle.next_dt(0.5, 0.03, 0.1, delta=0.1) == pytest.approx(0.05, rel=1e-15)
    assert oracle.next_dt(3.0, 0.06, 1.0) == pytest.approx(0.02, rel=1e-15)


def test_large_epsilon_is_the_fixed_step_scheme():
    # with eps huge every step is the cap, so the run is the fixed-step run
    rp, ci = W.random_regular(2000, 6, 5)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.12, "dt": 0.1, "seed": 9}
    seeds = W.seed_nodes(n, 10, 3)
    st0 = W.initial_state(n, seeds)
    a0 = np.zeros(n, np.float32)
    st, age, hist, dts = oracle.run_adaptive((rp, ci), model, st0, a0, 150, eps=1e9, dt_max=0.1)
    st_f, age_f, hist_f = oracle.run((rp, ci), model, st0, a0, 150)
    np.testing.assert_array_equal(dts, np.float64(0.1))
    np.testing.assert_array_equal(hist, hist_f)
    np.testing.assert_array_equal(st, st_f)
    np.testing.assert_array_equal(age, age_f)
    assert hist[-1, 0] < n - 50  # the epidemic moved


def test_constant_rates_under_a_varying_step():
    """E and I both exponential with rate g, beta = 0, every node seeded in E.
    Every node's rate is g while it is in E or I, so (with many nodes) the
    largest rate is g at every step: the first step is the cap dt_max and all
    later ones eps/g.  A node still in E after K steps survived K Bernoulli
    trials of probability exp(-g dt_k), so E_K ~ Binomial(N0, exp(-g T_K))
    with T_K the sum of the first K steps; a node is in I after K steps when
    it left E at some step j < K and survived the steps j+1 .. K-1 in I."""
    n0, g, eps, dt_max, K = 40_000, 0.5, 0.03, 0.1, 60
    rp = np.zeros(n0 + 1, np.int32)
    ci = np.zeros(0, np.int32)
    model = {"ei": ("exp", g), "ir": ("exp", g), "beta": 0.0, "dt": dt_max, "seed": 17}
    st0 = np.full(n0, 1, np.int32)
    _, _, hist, dts = oracle.run_adaptive((rp, ci), model, st0, np.zeros(n0, np.float32), K,
                                          eps=eps, dt_max=dt_max)
    assert dts[0] == dt_max
    np.testing.assert_allclose(dts[1:], eps / g, rtol=1e-15)
    a = np.exp(-g * dts)                      # per-step survival in a state
    for k in [5, 20, K]:
        pe = np.prod(a[:k])
        mean, sd = n0 * pe, math.sqrt(n0 * pe * (1 - pe))
        assert abs(hist[k - 1, 1] - mean) < 5 * sd, (k, hist[k - 1, 1], mean)
        pi = sum(np.prod(a[:j]) * (1 - a[j]) * np.prod(a[j + 1:k]) for j in range(k))
        mean, sd = n0 * pi, math.sqrt(n0 * pi * (1 - pi))
        assert abs(hist[k - 1, 2] - mean) < 5 * sd, (k, hist[k - 1, 2], mean)
    np.testing.assert_array_equal(hist.sum(1), n0)
    # a plausible slip (the first step also at eps/g) moves E_5 by about 10 sd
    pe_wrong = np.exp(-g * 5 * eps / g)
    assert abs(n0 * np.prod(a[:5]) - n0 * pe_wrong) > 8 * math.sqrt(n0 * pe_wrong * (1 - pe_wrong))


def test_step_after_an_idle_step_is_the_cap():
    # no E/I node and no pressure: every rate is 0, so every step is the cap
    rp, ci = W.random_regular(500, 4, 1)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 2}
    _, _, hist, dts = oracle.run_adaptive((rp, ci), model, np.zeros(n, np.int32),
                                          np.zeros(n, np.float32), 10, eps=0.03, dt_max=0.25)
    np.testing.assert_array_equal(dts, 0.25)
    np.testing.assert_array_equal(hist[:, 0], n)
