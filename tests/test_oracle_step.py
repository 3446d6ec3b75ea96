"""Pins for the oracle's whole tau-leap step (Algorithm 3, Eq. (influence),
Eq. (infectivity), Section "Bernoulli tau-leaping").

Each check compares the oracle with something other than itself:
  * pressure: brute force through a dense adjacency matrix (numpy);
  * the Markovian special case: exact binomial laws of the discrete scheme;
  * infection alone: the geometric survival law exp(-beta m k dt);
  * renewal holding times: the scheme's survival is the left Riemann product
    of exp(-h(n dt) dt), with h taken from scipy.stats pdf/sf (the hazard is
    read at the start-of-step age);
  * the whole epidemic on a complete graph: the age-structured discrete
    mean-field recursion of the same scheme (large-N limit);
  * the true continuous-time process: an exact event-driven simulation on a
    20-node graph, to which the scheme converges as dt -> 0;
  * the paper's printed epsilon-sweep row (coarse semantic check).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dense(rp, ci, w=None):
    n = len(rp) - 1
    A = np.zeros((n, n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            A[i, ci[e]] += 1.0 if w is None else float(w[e])
    return A


def binom_z(count, n, p):
    return (count - n * p) / math.sqrt(max(n * p * (1 - p), 1e-300))


# ---------------------------------------------------------------- pressure

def test_pressure_paper_csr_bruteforce(orc):
    g = json.load(open(os.path.join(GOLD, "paper_csr_example.json")))
    rp = np.array(g["row_ptr"], np.int32)
    ci = np.array(g["col_ind"], np.int32)
    A = dense(rp, ci)
    # all susceptible targets; each infected pattern of the five nodes
    beta = 0.37
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": beta, "dt": 0.1, "seed": 1}
    for mask in range(32):
        iota = np.array([(mask >> j) & 1 for j in range(5)], np.float64)
        st = np.zeros(5, np.int32)
        out = orc.step((rp, ci), model, st, np.zeros(5, np.float32), iota, 0)
        np.testing.assert_array_equal(out["lam"], beta * (A @ iota))
    # the highlighted row 2 reads col_ind[3..5] = {1, 3, 4}
    assert list(ci[rp[2]:rp[3]]) == [1, 3, 4]


def test_pressure_weighted_dense(orc):
    rng = np.random.default_rng(3)
    n = 60
    src = rng.integers(0, n, 400)
    dst = rng.integers(0, n, 400)
    rp, ci = W.csr_from_edges(n, src, dst, symmetric=False)
    w = rng.random(len(ci)).astype(np.float32)
    iota = rng.random(n)
    A = dense(rp, ci, w)
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": 1.0, "dt": 0.1, "seed": 1}
    out = orc.step((rp, ci, w), model, np.zeros(n, np.int32), np.zeros(n, np.float32), iota, 0)
    np.testing.assert_allclose(out["lam"], A @ iota, rtol=1e-14, atol=0)


def test_unit_weights_equal_null_weights(orc):
    rp, ci = W.random_regular(200, 6, 1)
    rng = np.random.default_rng(0)
    st = rng.integers(0, 4, 200).astype(np.int32)
    iota = (st == 2).astype(np.float64)
    age = rng.random(200).astype(np.float32) * 10
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.2, "dt": 0.1, "seed": 4}
    a = orc.step((rp, ci), model, st, age, iota, 7)
    b = orc.step((rp, ci, np.ones(len(ci), np.float32)), model, st, age, iota, 7)
    for k in ["state", "age", "iota", "counts", "lam", "q", "u"]:
        np.testing.assert_array_equal(a[k], b[k])


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("compact", [False, True])
def test_step_invariants(orc, compact):
    n = 3000
    rp, ci = W.random_regular(n, 10, 2)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 9}
    st0 = W.initial_state(n, W.seed_nodes(n, 30, 1))
    age0 = np.zeros(n, np.uint16 if compact else np.float32)
    st, age, _ = orc.run((rp, ci), model, st0, age0, 120, compact=compact)
    iota = (st == 2).astype(np.float64)
    out = orc.step((rp, ci), model, st, age, iota, 120, compact=compact)
    ns, na = out["state"], out["age"]
    d = ns - st
    assert set(np.unique(d)) <= {0, 1}                 # at most one transition per step
    assert np.all(ns[st == 3] == 3)                      # R absorbing
    assert np.all(out["lam"][st == 3] == 0.0)
    fired = d == 1
    assert np.all(na[fired] == 0)                        # renewal: age resets
    if compact:
        np.testing.assert_array_equal(na[~fired], np.minimum(age[~fired].astype(np.int64) + 1, 65535))
    else:
        np.testing.assert_array_equal(na[~fired], (age[~fired] + np.float32(0.1)).astype(np.float32))
    np.testing.assert_array_equal(out["iota"], (ns == 2).astype(np.float64))
    np.testing.assert_array_equal(out["counts"], np.bincount(ns, minlength=4))
    drew = out["lam"] > 0
    assert np.all(out["u"][~drew] == -1.0)
    np.testing.assert_array_equal(fired, drew & (out["u"] < out["q"]))
    # draws are the keyed uniforms of this step
    np.testing.assert_array_equal(out["u"][drew], orc.uniforms(9, np.flatnonzero(drew), 120, 0))
    # q = 1 - exp(-lambda dt)
    # (1 - exp(-x) in the test itself loses digits for small x, hence the absolute floor)
    np.testing.assert_allclose(out["q"], 1.0 - np.exp(-out["lam"] * 0.1), rtol=1e-12, atol=1e-15)


def test_step_nodes_and_run_agree_with_step(orc):
    n = 2000
    rp, ci = W.random_regular(n, 8, 4)
    model = {"ei": ("weibull", 2.0, 6.0), "ir": ("erlang", 3, 1.0), "beta": 0.25, "dt": 0.1,
             "seed": 2**40 + 5}
    st0 = W.initial_state(n, W.seed_nodes(n, 20, 2))
    st, age, _ = orc.run((rp, ci), model, st0, np.zeros(n, np.float32), 50, replica=3)
    iota = (st == 2).astype(np.float64)
    full = orc.step((rp, ci), model, st, age, iota, 50, replica=3)
    nodes = np.random.default_rng(1).choice(n, 300, replace=False)
    part = orc.step_nodes((rp, ci), model, st, age, iota, 50, nodes, replica=3)
    for k in ["state", "age", "lam", "q", "u"]:
        np.testing.assert_array_equal(part[k], full[k][nodes])
    # run(k steps) == k single steps with ping-pong infectivity
    s1, a1, h1 = orc.run((rp, ci), model, st0, np.zeros(n, np.float32), 60, replica=3)
    s2, a2 = st0.copy(), np.zeros(n, np.float32)
    io = (s2 == 2).astype(np.float64)
    for k in range(60):
        o = orc.step((rp, ci), model, s2, a2, io, k, replica=3)
        s2, a2, io = o["state"], o["age"], o["iota"]
        np.testing.assert_array_equal(o["counts"], h1[k])
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(a1, a2)


def test_compact_age_saturates(orc):
    rp = np.zeros(3, np.int32)
    ci = np.zeros(0, np.int32)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.0, "dt": 0.1, "seed": 0}
    st = np.array([0, 3], np.int32)
    out = orc.step((rp, ci), model, st, np.array([65534, 65535], np.uint16), np.zeros(2), 0,
                   compact=True)
    np.testing.assert_array_equal(out["age"], [65535, 65535])


# ---------------------------------------------------- Markovian closed forms

def test_markovian_limit_binomial_laws(orc):
    # exponential E and I, beta = 0, every node exposed, no edges: nodes are
    # independent, E_k ~ Bin(N, a^k) and I_k ~ Bin(N, (1-a)(b^k - a^k)/(b - a)),
    # a = exp(-gE dt), b = exp(-gI dt) (the discrete scheme, exact)
    n = 200_000
    gE, gI, dt = 1.0 / 3.0, 1.0 / 6.0, 0.1
    rp = np.zeros(n + 1, np.int32)
    ci = np.zeros(0, np.int32)
    model = {"ei": ("exp", gE), "ir": ("exp", gI), "beta": 0.0, "dt": dt, "seed": 77}
    st0 = np.ones(n, np.int32)
    _, _, h = orc.run((rp, ci), model, st0, np.zeros(n, np.float32), 100)
    a, b = math.exp(-gE * dt), math.exp(-gI * dt)
    for k in [1, 10, 50, 100]:
        pE = a**k
        pI = (1 - a) * (b**k - a**k) / (b - a)
        assert abs(binom_z(h[k - 1, 1], n, pE)) < 5
        assert abs(binom_z(h[k - 1, 2], n, pI)) < 5
        assert h[k - 1].sum() == n
    # the worked value quoted for this case: I_100/N = 0.30898 (discrete) vs 0.30640 (ODE)
    assert abs((1 - a) * (b**100 - a**100) / (b - a) - 0.30898) < 1e-5


def test_infection_only_geometric_survival(orc):
    # star centres (S) each fed by m permanently infectious leaves:
    # P(centre still S after k steps) = exp(-beta m dt k)
    stars, m = 40_000, 3
    rp, ci = W.star_forest(stars, m)
    n = len(rp) - 1
    st = np.full(n, 2, np.int32)
    st[::m + 1] = 0
    beta, dt = 0.2, 0.1
    model = {"ei": ("exp", 0.0), "ir": ("exp", 0.0), "beta": beta, "dt": dt, "seed": 5}
    _, _, h = orc.run((rp, ci), model, st, np.zeros(n, np.float32), 40)
    for k in [1, 5, 20, 40]:
        assert abs(binom_z(h[k - 1, 0], stars, math.exp(-beta * m * dt * k))) < 5
        assert h[k - 1, 2] == stars * m


@pytest.mark.parametrize("law", [W.LN_E, ("lognormal", math.log(2.0), 0.3),
                                 ("weibull", 2.0, 6.0), ("erlang", 3, 1.0)])
def test_renewal_survival_is_left_riemann_product(orc, law):
    # nodes exposed at age 0, beta = 0: P(still E after k steps) =
    # prod_{j<k} exp(-h(j dt) dt), hazard from scipy pdf/sf at the start-of-step age
    n, dt = 200_000, 0.5
    if law[0] == "lognormal":
        d = stats.lognorm(s=law[2], scale=math.exp(law[1]))
    elif law[0] == "weibull":
        d = stats.weibull_min(c=law[1], scale=law[2])
    else:
        d = stats.gamma(a=law[1], scale=1.0 / law[2])
    steps = 16
    tau = np.arange(steps) * dt
    h = np.zeros(steps)
    h[1:] = d.pdf(tau[1:]) / d.sf(tau[1:])
    surv = np.exp(-np.cumsum(h) * dt)
    rp = np.zeros(n + 1, np.int32)
    model = {"ei": law, "ir": ("exp", 0.0), "beta": 0.0, "dt": dt, "seed": 12}
    _, _, hist = orc.run((rp, np.zeros(0, np.int32)), model, np.ones(n, np.int32),
                         np.zeros(n, np.uint16), steps, compact=True)
    for k in range(1, steps + 1):
        assert abs(binom_z(hist[k - 1, 1], n, surv[k - 1])) < 5, k
    # a right-Riemann reading (hazard at the end-of-step age) is rejected
    surv_right = np.exp(-np.cumsum(d.pdf(tau + dt) / d.sf(tau + dt)) * dt)
    zs = [binom_z(hist[k - 1, 1], n, surv_right[k - 1]) for k in range(4, steps + 1)]
    assert max(abs(z) for z in zs) > 8


# ------------------------------------------------------------- mean field

def _mean_field(frac0, c, dt, steps, ei, ir):
    def qcurve(spec):
        d = stats.lognorm(s=spec[2], scale=math.exp(spec[1]))
        tau = np.arange(steps + 1) * dt
        h = np.zeros(steps + 1)
        h[1:] = d.pdf(tau[1:]) / d.sf(tau[1:])
        return -np.expm1(-h * dt)
    qE, qI = qcurve(ei), qcurve(ir)
    s, r = 1 - frac0, 0.0
    e = np.zeros(steps + 1)
    e[0] = frac0
    i = np.zeros(steps + 1)
    out = []
    for _ in range(steps):
        qs = -math.expm1(-c * i.sum() * dt)
        ne, ni = np.zeros_like(e), np.zeros_like(i)
        ne[0] = s * qs
        ne[1:] = e[:-1] * (1 - qE[:-1])
        ni[0] = (e * qE).sum()
        ni[1:] = i[:-1] * (1 - qI[:-1])
        r += (i * qI).sum()
        s -= s * qs
        e, i = ne, ni
        out.append((s, e.sum(), i.sum(), r))
    return np.array(out)


def test_complete_graph_mean_field(orc):
    N, c, dt, steps, ns = 300, 0.5, 0.1, 300, 15
    rp, ci = W.complete_graph(N)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": c / (N - 1), "dt": dt, "seed": 3}
    init = W.initial_state(N, np.arange(ns))
    H = np.array([orc.run((rp, ci), model, init, np.zeros(N, np.uint16), steps, replica=r,
                          compact=True)[2] / N for r in range(60)])
    ref = _mean_field(ns / N, c, dt, steps, W.LN_E, W.LN_I)
    mean, se = H.mean(0), H.std(0) / math.sqrt(len(H))
    for k in range(24, steps, 25):
        for comp in range(4):
            assert abs(mean[k, comp] - ref[k, comp]) < 3 * se[k, comp] + 0.01, (k, comp)


# --------------------------------------------------------- exact process

def test_converges_to_exact_process_small_graph(orc):
    # 20-node random 4-regular graph; exact event-driven simulation vs the
    # tau-leap at dt = 0.4 and 0.05.  The scheme's error is first order in dt:
    # large at 0.4, within noise at 0.05.
    n, T = 20, 60.0
    rp, ci = W.random_regular(n, 4, 5)
    beta = 0.15
    init = np.zeros(n, np.int32)
    init[0] = 1
    peaks, counts = orc.gillespie((rp, ci), W.LN_E, W.LN_I, beta, T, init, 1, 40_000)
    ex_ar = 1 - counts[:, 0] / n
    ex_pk = peaks / n
    res = {}
    for dt, reps in [(0.4, 12_000), (0.05, 6_000)]:
        model = {"ei": W.LN_E, "ir": W.LN_I, "beta": beta, "dt": dt, "seed": 1}
        steps = int(round(T / dt))
        pk = np.empty(reps)
        ar = np.empty(reps)
        for r in range(reps):
            _, _, h = orc.run((rp, ci), model, init, np.zeros(n, np.float32), steps, replica=r)
            pk[r] = h[:, 2].max() / n
            ar[r] = 1 - h[-1, 0] / n
        se_ar = math.sqrt(ar.var() / reps + ex_ar.var() / len(ex_ar))
        res[dt] = (ar.mean() - ex_ar.mean(), se_ar, pk.mean() - ex_pk.mean())
    bias_big, se_big, _ = res[0.4]
    bias_small, se_small, pk_small = res[0.05]
    assert abs(bias_big) > 4 * se_big                  # visible first-order error at dt = 0.4
    assert abs(bias_small) < 4 * se_small + abs(bias_big) * 0.05 / 0.4 * 1.5
    assert abs(bias_small) < abs(bias_big) / 2
    assert abs(pk_small) < 0.01


# ------------------------------------------------------- paper's numbers

def test_paper_epsilon_sweep_row_coarse(orc):
    g = json.load(open(os.path.join(GOLD, "paper_epsilon_sweep.json")))
    n = 1000
    EI = ("lognormal", math.log(4.0), math.sqrt(2 * math.log(5 / 4)))
    IR = ("lognormal", math.log(5.0), math.sqrt(2 * math.log(7.5 / 5)))
    rp, ci = W.erdos_renyi(n, 8.0, 0)
    init = W.initial_state(n, W.seed_nodes(n, 10, 1000))
    model = {"ei": EI, "ir": IR, "beta": 0.25, "dt": 0.1, "seed": 0}
    P, Rf = [], []
    for r in range(100):
        _, _, h = orc.run((rp, ci), model, init, np.zeros(n, np.float32), 500, replica=r)
        P.append(h[:, 2].max() / n)
        Rf.append(h[-1, 3] / n)
    # coarse: the paper's own graph instances and adaptive dt differ from ours
    assert abs(np.mean(P) - g["peak_I"]) < g["peak_I_ci95"] + 0.02
    assert abs(np.mean(Rf) - g["final_R"]) < g["final_R_ci95"] + 0.03
