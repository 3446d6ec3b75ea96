"""Pins of the oracle's Markovian engine step (Section "Markovian engine",
Algorithm "Markovian Engine: One Tau-Leaping Step").

The pieces are pinned one by one: the draws against the Philox already pinned
to numpy and rocRAND, the influence against a dense brute force, the step
size against its closed form in cases where each term of the minimum binds,
one step's transition counts against exact binomial laws (which also tell
1 - exp(-lambda tau) from lambda tau, and I -> S from I -> R), SIS against
the endemic level of the complete graph, and whole SEIR/SIR epidemics against
the exact event-driven simulator of the same continuous-time process.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

BASE = {"beta": 0.3, "sigma": 0.5, "gamma": 0.2, "theta": 0.01, "p_max": 0.1, "tau_max": 1.0, "seed": 7}


def test_draws_are_the_pinned_philox_uniforms():
    rp, ci = W.random_regular(500, 4, 3)
    n = len(rp) - 1
    st = np.full(n, 2, np.int32)          # every node infectious: every node draws
    m = dict(BASE, model="sir", seed=0x0123456789ABCDEF)
    out = oracle.markov_step((rp, ci), m, st, 41)
    np.testing.assert_array_equal(out["u"], oracle.uniforms(m["seed"], np.arange(n), 41, 0))


def test_influence_is_the_count_of_infectious_in_neighbours():
    rng = np.random.default_rng(1)
    n = 300
    A = (rng.random((n, n)) < 0.04).astype(np.int64)   # A[i, j] = 1: edge j -> i
    np.fill_diagonal(A, 0)
    rp = np.concatenate([[0], np.cumsum(A.sum(1))]).astype(np.int32)
    ci = np.concatenate([np.flatnonzero(A[i]) for i in range(n)]).astype(np.int32)
    st = rng.integers(0, 4, n).astype(np.int32)
    np.testing.assert_array_equal(oracle.markov_influence((rp, ci), st), A @ (st == 2))


def test_step_size_rule():
    rp, ci = W.random_regular(1000, 6, 2)
    n = len(rp) - 1
    g = (rp, ci)
    # no positive rate: the cap
    tau, L, M = oracle.markov_tau(g, dict(BASE, model="seir"), np.zeros(n, np.int32))
    assert (tau, L, M) == (1.0, 0.0, 0.0)
    # only infectious nodes, no susceptible: Lambda = gamma nI, max = gamma
    st = np.full(n, 3, np.int32)
    st[:40] = 2
    for theta, pmax, tmax, want in [(0.001, 0.1, 1.0, 0.001 * n / (0.2 * 40)),  # theta N / Lambda binds
                                    (0.5, 0.1, 1.0, 0.1 / 0.2),                 # p_max / max binds
                                    (0.5, 0.9, 0.7, 0.7)]:                      # the cap binds
        m = dict(BASE, model="sir", theta=theta, p_max=pmax, tau_max=tmax)
        tau, L, M = oracle.markov_tau(g, m, st)
        assert L == pytest.approx(0.2 * 40, rel=1e-15) and M == 0.2
        assert tau == pytest.approx(want, rel=1e-15)
    # susceptible rates: beta * influence, summed and maximised over all nodes
    st = np.zeros(n, np.int32)
    st[::7] = 2
    infl = oracle.markov_influence(g, st)
    m = dict(BASE, model="seir")
    tau, L, M = oracle.markov_tau(g, m, st)
    lam = np.where(st == 0, 0.3 * infl, 0.0) + np.where(st == 2, 0.2, 0.0)
    assert L == pytest.approx(lam.sum(), rel=1e-13) and M == pytest.approx(lam.max(), rel=1e-15)
    assert tau == pytest.approx(min(0.01 * n / lam.sum(), 0.1 / lam.max(), 1.0), rel=1e-13)


@pytest.mark.parametrize("model,start,rate,dest", [("seir", 1, "sigma", 2), ("sir", 2, "gamma", 3),
                                                   ("sis", 2, "gamma", 0)])
def test_one_step_counts_are_binomial(model, start, rate, dest):
    """Every node in one compartment with no susceptible neighbour: the
    number that leave is Binomial(n, 1 - exp(-r tau)) with tau from the rule,
    and they land in the model's next compartment."""
    n = 200_000
    rp = np.zeros(n + 1, np.int32)           # no edges: no infection
    ci = np.zeros(0, np.int32)
    m = dict(BASE, model=model, theta=1.0, p_max=0.3, tau_max=5.0, seed=99)
    st = np.full(n, start, np.int32)
    out = oracle.markov_step((rp, ci), m, st, 3)
    r = m[rate]
    tau = min(1.0 * n / (r * n), 0.3 / r, 5.0)
    assert out["tau"] == pytest.approx(tau, rel=1e-15)
    moved = int((out["state"] == dest).sum())
    assert moved + int((out["state"] == start).sum()) == n
    p = -math.expm1(-r * tau)
    sd = math.sqrt(n * p * (1 - p))
    assert abs(moved - n * p) < 5 * sd, (moved, n * p, sd)
    assert abs(n * r * tau - n * p) > 8 * sd       # lambda * tau instead of 1 - exp(-lambda tau)
    assert out["events"] == moved


def test_sis_reaches_the_complete_graph_endemic_level():
    """SIS on the complete graph K_n: the quasi-stationary infected fraction
    is 1 - gamma / (beta (n - 1)) to first order in 1/n (mean field is exact
    on K_n as n grows); with R0 = 2 that is one half."""
    n = 1500
    rp = (np.arange(n + 1) * (n - 1)).astype(np.int32)
    ci = np.concatenate([np.delete(np.arange(n), i) for i in range(n)]).astype(np.int32)
    gamma = 0.25
    beta = 2.0 * gamma / (n - 1)
    m = dict(BASE, model="sis", beta=beta, gamma=gamma, theta=0.01, p_max=0.1, tau_max=1.0, seed=5)
    st = np.zeros(n, np.int32)
    st[:50] = 2
    _, hist, taus, _ = oracle.markov_run((rp, ci), m, st, 3000)
    t = np.cumsum(taus)
    late = t > t[-1] / 2
    frac = float((hist[late, 2] * taus[late]).sum() / taus[late].sum() / n)
    assert abs(frac - 0.5) < 0.02, frac
    assert np.all(hist[:, 3] == 0)       # SIS never removes anyone
    # an I -> R slip would end the epidemic instead
    _, hist_sir, _, _ = oracle.markov_run((rp, ci), dict(m, model="sir"), st, 3000)
    assert hist_sir[-1, 2] < 0.05 * n


@pytest.mark.parametrize("model", ["seir", "sir"])
def test_epidemic_matches_the_exact_simulator(model):
    """The tau-leap at the paper's defaults (theta = 0.01, p_max = 0.1)
    against the exact event-driven simulation of the same Markovian process
    (exponential holding times; SIR as SEIR with an exposed stage of mean
    1e-6 days): final attack rate and peak prevalence over 60 runs each,
    within 3 standard errors plus 0.01."""
    rp, ci = W.erdos_renyi(1000, 8.0, 12)
    n = len(rp) - 1
    beta, sigma, gamma = 0.25, 0.4, 0.15
    seeds = W.seed_nodes(n, 10, 4)
    st0 = np.zeros(n, np.int32)
    st0[seeds] = 2
    reps = 60
    t_end = 150.0
    ei = ("exp", sigma) if model == "seir" else ("exp", 1e6)
    peaks, counts = oracle.gillespie((rp, ci), ei, ("exp", gamma), beta, t_end, st0, 11, reps)
    ex = np.stack([counts[:, 3] / n, peaks / n], 1)
    tl = []
    for r in range(reps):
        m = {"model": model, "beta": beta, "sigma": sigma, "gamma": gamma, "theta": 0.01, "p_max": 0.1,
             "tau_max": 1.0, "seed": 1000 + r}
        st, hist, taus, _ = oracle.markov_run((rp, ci), m, st0, 4000)
        T = np.cumsum(taus)
        assert T[-1] > t_end or hist[-1, 1] + hist[-1, 2] == 0
        k = min(int(np.searchsorted(T, t_end)), len(T) - 1)
        tl.append((hist[k, 3] / n, hist[: k + 1, 2].max() / n))
    tl = np.array(tl)
    for j, name in enumerate(["attack rate", "peak"]):
        se = math.sqrt(ex[:, j].var(ddof=1) / reps + tl[:, j].var(ddof=1) / reps)
        assert abs(ex[:, j].mean() - tl[:, j].mean()) < 3 * se + 0.01, (name, ex[:, j].mean(), tl[:, j].mean(), se)
    assert ex[:, 0].mean() > 0.3
