"""Pins of the oracle's shedding profiles s(tau) (Eq. (infectivity): the
infectivity of an infectious source is beta s(tau_j); Table "agedep_overhead"
uses a hazard-shaped profile).

The profile's values are pinned to scipy's densities and hazards.  Its use in
the step is pinned by closed-form laws: on a star whose hub stays infectious,
and whose leaves are susceptible and never become infectious, a leaf escapes
K steps with probability exp(-beta dt sum_k w s(tau_k)), where tau_k is the
hub's age at the start of step k.  The hub's age is known exactly, so
E_K ~ Binomial(M, 1 - exp(...)).  Each case also checks that a plausible slip
(the age after the step instead of before it, a dropped weight) would move
the count by many standard deviations.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W

TAUS = np.array([0.0, 1e-3, 0.05, 0.1, 0.5, 1.0, 2.5, 7.0, 20.0])


def scipy_law(spec):
    kind = spec[0]
    if kind == "exp":
        return stats.expon(scale=1.0 / spec[1])
    if kind == "lognormal":
        return stats.lognorm(s=spec[2], scale=math.exp(spec[1]))
    if kind == "weibull":
        return stats.weibull_min(c=spec[1], scale=spec[2])
    return stats.gamma(a=spec[1], scale=1.0 / spec[2])


LAWS = [("exp", 0.7), ("lognormal", math.log(3.0), 0.5), ("lognormal", 0.2, 1.1), ("weibull", 1.0, 2.0),
        ("weibull", 2.5, 4.0), ("erlang", 1, 0.8), ("erlang", 3, 1.2), ("erlang", 12, 2.5)]


@pytest.mark.parametrize("law", LAWS, ids=[f"{l[0]}-{i}" for i, l in enumerate(LAWS)])
def test_density_matches_scipy(law):
    got = oracle.density(law, TAUS)
    want = scipy_law(law).pdf(TAUS)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-300)


def test_infectivity_values_per_mode():
    rng = np.random.default_rng(3)
    n = 400
    st = rng.integers(0, 4, n).astype(np.int32)
    age = rng.uniform(0.0, 9.0, n).astype(np.float32)
    base = {"ei": ("exp", 1.0), "ir": ("exp", 1.0), "beta": 0.1, "dt": 0.1}
    isI = st == 2
    law = ("lognormal", math.log(2.0), 0.6)
    np.testing.assert_array_equal(oracle.infectivity(base, st, age), isI.astype(float))
    got = oracle.infectivity(dict(base, shed=("density", law, 2.5)), st, age)
    np.testing.assert_allclose(got, np.where(isI, 2.5 * scipy_law(law).pdf(age.astype(np.float64)), 0.0),
                               rtol=1e-12)
    wb = ("weibull", 2.0, 3.0)
    d = scipy_law(wb)
    got = oracle.infectivity(dict(base, shed=("hazard", wb, 0.4)), st, age)
    a64 = age.astype(np.float64)
    np.testing.assert_allclose(got, np.where(isI, 0.4 * d.pdf(a64) / d.sf(a64), 0.0), rtol=1e-12)
    # compact storage: ages are whole steps (tau = n * dt) and the stored
    # value is binary16 (numpy's float64 -> float16 conversion rounds to
    # nearest even)
    steps = rng.integers(0, 300, n).astype(np.uint16)
    got = oracle.infectivity(dict(base, dt=0.2, shed=("density", law, 1.0)), st, steps, compact=True)
    want = scipy_law(law).pdf(steps * 0.2).astype(np.float16).astype(np.float64)
    np.testing.assert_allclose(got, np.where(isI, want, 0.0), rtol=1e-12)
    np.testing.assert_array_equal(oracle.infectivity(base, st, steps, compact=True), isI.astype(float))


def test_binary16_rounding_matches_numpy():
    # the oracle's storage rounding of compact infectivity values against
    # numpy's conversion: random magnitudes over the whole range, exact
    # midpoints (ties go to even), the subnormal range, the overflow edge
    rng = np.random.default_rng(11)
    x = np.exp(rng.uniform(math.log(1e-9), math.log(1e6), 200_000))
    x = np.concatenate([x, -x[:1000]])
    h = np.arange(0, 0x7BFF, dtype=np.uint16).view(np.float16).astype(np.float64)
    mid = (h[:-1] + h[1:]) / 2.0                          # exact in float64
    edge = np.array([0.0, -0.0, 2.0**-24, 2.0**-25, 3 * 2.0**-26, 2.0**-14, 65504.0, 65519.99, 65520.0,
                     65536.0, 1e9, np.inf, -np.inf])
    for v in (x, mid, edge):
        with np.errstate(over="ignore"):  # (the overflow edge: float16 infinity is expected)
            want = v.astype(np.float16).astype(np.float64)
        np.testing.assert_array_equal(oracle.binary16(v), want)
    assert np.isnan(oracle.binary16(np.array([np.nan]))[0])


def test_write_back_uses_the_age_after_the_step():
    """The step's output infectivity is s(tau') 1{X' = I}: ages advanced by dt
    for nodes that stayed infectious, 0 for nodes that just became
    infectious (exponential density: s(0) = A * rate > 0)."""
    rp, ci = W.random_regular(3000, 6, 2)
    n = len(rp) - 1
    rng = np.random.default_rng(5)
    st = rng.choice(4, n, p=[0.5, 0.2, 0.2, 0.1]).astype(np.int32)
    age = rng.uniform(0.0, 5.0, n).astype(np.float32)
    law = ("exp", 0.9)
    model = {"ei": ("exp", 3.0), "ir": ("exp", 0.5), "beta": 0.4, "dt": 0.25, "seed": 8,
             "shed": ("density", law, 1.7)}
    io = oracle.infectivity(model, st, age)
    out = oracle.step((rp, ci), model, st, age, io, 0)
    nst, nage = out["state"], out["age"]
    isI = nst == 2
    want = np.where(isI, 1.7 * 0.9 * np.exp(-0.9 * nage.astype(np.float64)), 0.0)
    np.testing.assert_allclose(out["iota"], want, rtol=1e-13)
    fresh = isI & (st == 1)
    assert fresh.sum() > 50 and np.all(nage[fresh] == 0)
    np.testing.assert_allclose(out["iota"][fresh], 1.7 * 0.9, rtol=1e-15)
    stayed = isI & (st == 2)
    assert stayed.sum() > 50
    np.testing.assert_array_equal(nage[stayed], (age[stayed] + np.float32(0.25)).astype(np.float32))


def star(n_hubs, m, weights=None):
    """Hubs 0..n_hubs-1 with no incoming edges; leaves n_hubs.. each with one
    incoming edge from every hub (in hub order)."""
    rp = np.concatenate([np.zeros(n_hubs, np.int64), np.arange(m + 1) * n_hubs]).astype(np.int32)
    ci = np.tile(np.arange(n_hubs), m).astype(np.int32)
    if weights is None:
        return rp, ci
    return rp, ci, np.tile(np.asarray(weights, np.float32), m)


def hub_ages(a0, dt, k):
    """The hub's float32 ages at the start of steps 0..k (it never fires)."""
    out = [np.float32(a0)]
    for _ in range(k):
        out.append(np.float32(out[-1] + np.float32(dt)))
    return np.array(out, dtype=np.float64)


def binomial_check(count, m, p, label):
    mean, sd = m * p, math.sqrt(m * p * (1 - p))
    assert abs(count - mean) < 5 * sd, (label, count, mean, sd)
    return sd


def test_star_density_profile():
    m, beta, dt = 50_000, 0.5, 0.1
    law = ("lognormal", math.log(0.6), 0.4)
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": beta, "dt": dt, "seed": 21,
             "shed": ("density", law, 1.0)}
    rp, ci = star(1, m)
    st = np.zeros(m + 1, np.int32)
    st[0] = 2
    age = np.full(m + 1, 3.0, np.float32)   # leaves: an age far from the hub's
    age[0] = 0.05
    K = 25
    _, _, hist = oracle.run((rp, ci), model, st, age, K)
    ages = hub_ages(0.05, dt, K)
    f = scipy_law(law).pdf
    for k in [3, 10, 25]:
        p = 1 - math.exp(-beta * dt * f(ages[:k]).sum())
        sd = binomial_check(hist[k - 1, 1], m, p, k)
        if k == 3:
            # the age after each step instead of the age before it
            p_late = 1 - math.exp(-beta * dt * f(ages[1:k + 1]).sum())
            assert abs(m * p_late - m * p) > 8 * sd
            # the leaf's own age instead of the hub's
            p_tgt = 1 - math.exp(-beta * dt * f(hub_ages(3.0, dt, k)[:k]).sum())
            assert abs(m * p_tgt - m * p) > 8 * sd
    np.testing.assert_array_equal(hist[:, 2], 1)   # the hub stays infectious
    np.testing.assert_array_equal(hist[:, 3], 0)


def test_two_weighted_hubs_hazard_profile():
    m, beta, dt = 40_000, 0.3, 0.1
    law = ("weibull", 2.5, 1.5)
    w = [0.7, 1.9]
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": beta, "dt": dt, "seed": 4,
             "shed": ("hazard", law, 0.8)}
    g = star(2, m, w)
    st = np.zeros(m + 2, np.int32)
    st[:2] = 2
    age = np.zeros(m + 2, np.float32)
    age[0], age[1] = 0.3, 1.2
    K = 15
    _, _, hist = oracle.run(g, model, st, age, K)
    d = scipy_law(law)
    h = lambda t: 0.8 * d.pdf(t) / d.sf(t)
    a0, a1 = hub_ages(0.3, dt, K), hub_ages(1.2, dt, K)
    for k in [5, 15]:
        tot = w[0] * h(a0[:k]).sum() + w[1] * h(a1[:k]).sum()
        p = 1 - math.exp(-beta * dt * tot)
        sd = binomial_check(hist[k - 1, 1], m, p, k)
        p_now = 1 - math.exp(-beta * dt * (h(a0[:k]).sum() + h(a1[:k]).sum()))   # weights dropped
        assert abs(m * p_now - m * p) > 8 * sd
        p_swap = 1 - math.exp(-beta * dt * (w[1] * h(a0[:k]).sum() + w[0] * h(a1[:k]).sum()))
        assert abs(m * p_swap - m * p) > 8 * sd


def test_star_compact_ages():
    """Compact storage: ages are whole steps n, tau = n dt."""
    m, beta, dt = 50_000, 0.6, 0.2
    law = ("erlang", 3, 2.0)
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": beta, "dt": dt, "seed": 33,
             "shed": ("density", law, 1.5)}
    rp, ci = star(1, m)
    st = np.zeros(m + 1, np.int32)
    st[0] = 2
    age = np.full(m + 1, 40, np.uint16)
    age[0] = 2
    K = 12
    _, ag, hist = oracle.run((rp, ci), model, st, age, K, compact=True)
    assert ag[0] == 2 + K
    # the stored values are binary16 (compact storage)
    f = lambda t: (1.5 * scipy_law(law).pdf(t)).astype(np.float16).astype(np.float64)
    for k in [4, 12]:
        taus = (2 + np.arange(k)) * dt
        p = 1 - math.exp(-beta * dt * f(taus).sum())
        sd = binomial_check(hist[k - 1, 1], m, p, k)
        if k == 4:   # (on the rising flank of the profile)
            p_late = 1 - math.exp(-beta * dt * f(taus + dt).sum())
            assert abs(m * p_late - m * p) > 8 * sd


def test_unit_exponential_hazard_profile_is_constant_shedding():
    """s = 1 * h of an exponential law with rate 1 is s == 1: same trajectory."""
    rp, ci = W.random_regular(2000, 8, 9)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.15, "dt": 0.1, "seed": 12}
    seeds = W.seed_nodes(n, 20, 4)
    st0, a0 = W.initial_state(n, seeds), np.zeros(n, np.float32)
    ref = oracle.run((rp, ci), model, st0, a0, 120)
    alt = oracle.run((rp, ci), dict(model, shed=("hazard", ("exp", 1.0), 1.0)), st0, a0, 120)
    for x, y in zip(ref, alt):
        np.testing.assert_array_equal(x, y)
    assert ref[2][-1, 0] < n - 100
    # a profile that actually varies changes the trajectory
    var = oracle.run((rp, ci), dict(model, shed=("density", ("lognormal", math.log(3.0), 0.5), 3.0)),
                     st0, a0, 120)
    assert not np.array_equal(ref[2], var[2])
