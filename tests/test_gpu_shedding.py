"""Age-dependent shedding on the GPU (Eq. (infectivity) with a profile s(tau);
Table "agedep_overhead") against the FP64 oracle.

The device profile is compared value by value with the oracle's density and
hazard.  One step from a given state is compared node by node (states,
ages, rates), both right after a state load (values rebuilt from the state)
and one step later (values written by the step kernel itself).  A unit
exponential hazard profile (s == 1 exactly) must reproduce the
constant-shedding trajectory bit for bit on every kernel variant.

Tolerances.  s(tau) is evaluated in FP32 with float-float exponents; its
relative error against FP64 stays below PROFILE_TOL (a few ulp of the final
exp, division and scale).  The Weibull density holds one exponent term that
is itself an FP32 exponential, w = (tau / scale)^shape: its rounding
(<= 2 ulp) moves the exponent by up to 2^-22 w, so there the bound grows by
that much (w ~ 70 before the density leaves the FP32 range).  A pressure
sums such values in FP32, so S rates agree to RATE_TOL, and a draw may flip
where |u - q| is within GUARD_REL * q of the threshold.  Compact storage keeps
the values in binary16 on both sides (the oracle rounds its FP64 value, the
step its FP32 one): where the FP32 value falls within its error of a binary16
rounding boundary the two stored values differ by one unit in the last place
(2^-11 relative), and since a pressure sums non-negative terms, it then moves
by at most 2^-11 relative: COMPACT_TOL for rates and the guard band.
"""
import math
import zlib

import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W
from _parity import check_mismatch_budget

pytestmark = pytest.mark.gpu

PROFILE_TOL = 1e-5
RATE_TOL = 2e-5
GUARD_REL = 5e-5
COMPACT_TOL = 2.0**-11 + RATE_TOL
FLOOR = 1e-30

SMALL = W.WORKLOADS["regular10_n1e4"]

SHEDS = {
    "ln-density": ("density", ("lognormal", math.log(3.0), 0.5), 5.0),
    "wb-density": ("density", ("weibull", 2.2, 4.0), 4.0),
    "wb1-density": ("density", ("weibull", 1.0, 3.0), 3.0),
    "erl-density": ("density", ("erlang", 3, 0.8), 6.0),
    "erl1-density": ("density", ("erlang", 1, 0.5), 2.0),
    "exp-density": ("density", ("exp", 0.4), 2.0),
    "ln-hazard": ("hazard", W.LN_I, 1.0),
    "wb-hazard": ("hazard", ("weibull", 2.0, 5.0), 0.7),
    "erl-hazard": ("hazard", ("erlang", 4, 1.0), 1.3),
}


def oracle_profile(shed, tau):
    form, law, scale = shed
    f = oracle.density(law, tau) if form == "density" else oracle.hazard(law, tau)
    return scale * f


def profile_tol(shed, tau):
    form, law, _ = shed
    tol = np.full(len(tau), PROFILE_TOL)
    if form == "density" and law[0] == "weibull":
        tol += 2.0**-22 * (np.asarray(tau, np.float64) / law[2]) ** law[1]
    return tol


def check_profile(got, want, tol, label):
    got = np.asarray(got, np.float64)
    big = want >= FLOOR
    rel = np.abs(got[big] - want[big]) / want[big]
    worst = float((rel / tol[big]).max()) if rel.size else 0.0
    print(f"[profile] {label}: worst relative error {float(rel.max()):.2e}, {worst:.2f} of the bound")
    assert worst <= 1.0, (label, worst)
    assert np.all(np.abs(got[~big]) <= 1e-29), label
    return worst


@pytest.mark.parametrize("name", list(SHEDS))
def test_device_profile_matches_oracle(name):
    shed = SHEDS[name]
    # FP32 days: every age a run of 400 steps of 0.1 accumulates, plus random ones
    ages = [np.float32(0.0)]
    for _ in range(400):
        ages.append(np.float32(ages[-1] + np.float32(0.1)))
    rng = np.random.default_rng(1)
    a = np.concatenate([np.array(ages, np.float32), rng.uniform(0, 30, 5000).astype(np.float32)])
    tau = a.astype(np.float64)
    check_profile(fs.fs_eval_shedding(shed, a), oracle_profile(shed, tau), profile_tol(shed, tau), f"{name} days")
    # compact storage: whole steps of dt
    for dt in [0.1, 0.25]:
        n = np.arange(0, 2000, dtype=np.uint16)
        check_profile(fs.fs_eval_shedding(shed, n, fs.FS_STORAGE_COMPACT, dt),
                      oracle_profile(shed, n * dt), profile_tol(shed, n * dt), f"{name} steps dt={dt}")


def compare_step(gst, gage, grates, ora, label, compact=False):
    """Node-by-node check of one step; returns the number of guard-band flips."""
    guard = COMPACT_TOL if compact else GUARD_REL
    mism = np.flatnonzero(gst != ora["state"])
    bad = [int(i) for i in mism if not (ora["u"][i] >= 0 and abs(ora["u"][i] - ora["q"][i]) < guard * ora["q"][i] + 1e-6)]
    assert not bad, f"{label}: {len(bad)} mismatches outside the guard band, first {bad[:5]}"
    same = gst == ora["state"]
    np.testing.assert_array_equal(gage[same], ora["age"][same], err_msg=label)
    g = grates.astype(np.float64)
    o = ora["lam"]
    big = o >= FLOOR
    rel = np.abs(g[big] - o[big]) / o[big]
    assert rel.max() <= (COMPACT_TOL if compact else RATE_TOL), (label, float(rel.max()))
    assert np.all(np.abs(g[~big]) <= 1e-29), label
    return len(mism)


def random_state(n, compact, rng):
    st = rng.choice(4, n, p=[0.55, 0.12, 0.23, 0.10]).astype(np.int32)
    if compact:
        age = rng.integers(0, 120, n).astype(np.uint16)
    else:
        age = (rng.integers(0, 120, n) * np.float32(0.1)).astype(np.float32)
    return st, age


GRAPHS = {}


def graph(name):
    if name not in GRAPHS:
        if name == "regular":
            rp, ci = W.workload_graph(SMALL["graph"])
            GRAPHS[name] = (rp, ci, None)
        elif name == "ba":
            rp, ci = W.barabasi_albert(20_000, 5, 3)
            GRAPHS[name] = (rp, ci, None)
        else:
            rp, ci = W.random_regular(12_000, 7, 4)
            w = np.random.default_rng(2).uniform(0.2, 1.8, len(ci)).astype(np.float32)
            GRAPHS[name] = (rp, ci, w)
    return GRAPHS[name]


CASES = [
    ("regular", "resident", False, "ln-density"),
    ("regular", "summary", False, "wb-density"),
    ("regular", "stream", True, "erl-density"),
    ("regular", "resident", True, "ln-hazard"),
    ("ba", "resident", False, "ln-density"),
    ("ba", "stream", False, "exp-density"),
    ("ba", "summary", True, "wb-hazard"),
    ("weighted", "resident", False, "erl1-density"),
    ("weighted", "stream", True, "ln-density"),
]
VARIANTS = {"stream": fs.VARIANT_STREAM, "resident": fs.VARIANT_RESIDENT, "summary": fs.VARIANT_SUMMARY}


@pytest.mark.parametrize("gname,variant,compact,shed", CASES,
                         ids=["-".join([c[0], c[1], "compact" if c[2] else "fp32", c[3]]) for c in CASES])
def test_two_steps_match_the_oracle(gname, variant, compact, shed):
    rp, ci, w = graph(gname)
    n = len(rp) - 1
    gtuple = (rp, ci) if w is None else (rp, ci, w)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.2, "dt": 0.1, "seed": 77, "shed": SHEDS[shed]}
    rng = np.random.default_rng(zlib.crc32(f"{gname}/{variant}/{compact}/{shed}".encode()))
    storage = fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32
    mism, total = 0, 0
    with fs.Graph(rp, ci, w) as g:
        sim = fs.Sim.from_model(g, model, storage=storage, record_rates=True, variant=VARIANTS[variant])
        try:
            for k in [0, 37]:
                st, age = random_state(n, compact, rng)
                sim.set_state(st, age, 0, step_index=k)
                for j in range(2):
                    # step k+j from the GPU's own state: j = 0 reads values rebuilt
                    # after the load, j = 1 the values the step kernel wrote
                    cur_st, cur_age, kk = sim.get_state(0)
                    assert kk == k + j
                    iota = oracle.infectivity(model, cur_st, cur_age, compact=compact)
                    ora = oracle.step(gtuple, model, cur_st, cur_age, iota, k + j, compact=compact)
                    sim.step(1)
                    gst, gage, _ = sim.get_state(0)
                    mism += compare_step(gst, gage, sim.rates(0), ora, f"k={k + j}", compact)
                    total += n
                    assert ora["lam"][cur_st == 0].max() > 0
        finally:
            sim.close()
    check_mismatch_budget(mism, total, "shedding steps")


@pytest.mark.parametrize("gname", ["regular", "ba", "weighted"])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_unit_exponential_hazard_profile_equals_constant_shedding(gname, variant):
    rp, ci, w = graph(gname)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.15, "dt": 0.1, "seed": 5}
    seeds = W.seed_nodes(n, 30, 2)
    out = []
    with fs.Graph(rp, ci, w) as g:
        for shed in [None, ("hazard", ("exp", 1.0), 1.0)]:
            sim = fs.Sim.from_model(g, dict(model, shed=shed), variant=VARIANTS[variant], replicas=2,
                                    steps_per_graph=20)
            sim.seed(seeds)
            sim.step(150)
            out.append([(*sim.get_state(r)[:2], sim.history(0, 150, r)) for r in range(2)])
            sim.close()
    for a, b in zip(out[0], out[1]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    assert out[0][0][2][-1, 0] < n - 100   # the epidemic moved


PACKED_CASES = [c for c in CASES if c[0] != "weighted"]


@pytest.mark.parametrize("gname,variant,compact,shed", PACKED_CASES,
                         ids=["-".join([c[0], c[1], "compact" if c[2] else "fp32", c[3]]) for c in PACKED_CASES])
def test_packed_columns_with_shedding(gname, variant, compact, shed):
    """Single-replica sims of unweighted graphs take packed columns with
    age-dependent shedding too: the trajectory of 32-bit columns, bit for
    bit (the latter are checked against the oracle above)."""
    rp, ci, _ = graph(gname)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 5, "shed": SHEDS[shed]}
    storage = fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32
    seeds = W.seed_nodes(n, 25, 2)
    out = []
    with fs.Graph(rp, ci) as g:
        for cols in (fs.FS_COLUMNS_AUTO, fs.FS_COLUMNS_PLAIN):
            with fs.Sim.from_model(g, model, variant=VARIANTS[variant], storage=storage, steps_per_graph=25,
                                   history_len=150, columns=cols) as sim:
                out.append(sim.column_bits())
                sim.seed(seeds)
                sim.step(150)
                out.append((*sim.get_state(0)[:2], sim.history(0, 150)))
    assert out[0] == 20 and out[2] == 32
    for x, y in zip(out[1], out[3]):
        np.testing.assert_array_equal(x, y)
    assert out[1][2][-1, 0] < n - 75   # the epidemic moved beyond the 25 seeds


def test_shedding_changes_the_epidemic_as_the_oracle_does():
    """Replicas 0..7 of one GPU sim against oracle runs of the same replicas:
    final attack rates and peak prevalence agree within 3 standard errors
    (the draws are the same streams, so they agree far more closely unless
    the profile is misapplied)."""
    rp, ci, _ = graph("regular")
    n = len(rp) - 1
    shed = SHEDS["ln-density"]
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.08, "dt": 0.1, "seed": 31, "shed": shed}
    seeds = W.seed_nodes(n, 20, 9)
    steps, R = 300, 8
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, model, replicas=R, steps_per_graph=50)
        sim.seed(seeds)
        sim.step(steps)
        gh = [sim.history(0, steps, r) for r in range(R)]
        sim.close()
    oh = [oracle.run((rp, ci), model, W.initial_state(n, seeds), np.zeros(n, np.float32), steps,
                     replica=r)[2] for r in range(R)]
    stats = lambda h: (h[:, 2].max() / n, 1 - h[-1, 0] / n)
    a = np.array([stats(h) for h in gh])
    b = np.array([stats(h) for h in oh])
    for j in range(2):
        se = math.sqrt(a[:, j].var(ddof=1) / R + b[:, j].var(ddof=1) / R) + 1e-12
        assert abs(a[:, j].mean() - b[:, j].mean()) < 3 * se, (j, a[:, j], b[:, j])
    assert a[:, 1].mean() > 0.08
    # the constant profile with the same beta gives a different epidemic
    hc = oracle.run((rp, ci), dict(model, shed=None), W.initial_state(n, seeds), np.zeros(n, np.float32),
                    steps)[2]
    assert abs(stats(hc)[1] - a[:, 1].mean()) > 0.15


def test_shedding_rejections():
    rp, ci, _ = graph("regular")
    m = dict(SMALL["model"], shed=SHEDS["ln-density"])
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, m, variant=fs.VARIANT_STREAM)
        with fs.Batch() as b:
            with pytest.raises(fs.FsError):
                b.add(sim)
        sim.close()
        with fs.Server() as sv:
            with pytest.raises(fs.FsError):
                fs.fs_server_submit(sv.handle, g.handle,
                                    fs.make_params(m["ei"], m["ir"], 0.1, 0.1, 1, 1, shed=m["shed"]), 10, [0])
        for bad in [("density", ("weibull", 0.5, 2.0), 1.0), ("hazard", ("exp", 1.0), -1.0)]:
            with pytest.raises(fs.FsError) as ei:
                fs.Sim.from_model(g, dict(m, shed=bad))
            assert ei.value.status == 1


@pytest.mark.parametrize("gname", ["regular", "weighted", "ba"])
def test_variants_identical_with_shedding(gname):
    """Every kernel variant sums the same terms in the same order, also when
    rows have many infectious sources (half the nodes infectious here, so
    many rows exceed the first few sources a pass loads at once)."""
    rp, ci, w = graph(gname)
    n = len(rp) - 1
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.05, "dt": 0.1, "seed": 3,
             "shed": ("density", ("lognormal", math.log(3.0), 0.5), 5.0)}
    rng = np.random.default_rng(17)
    st = rng.choice(4, n, p=[0.4, 0.05, 0.5, 0.05]).astype(np.int32)
    age = (rng.integers(0, 80, n) * np.float32(0.1)).astype(np.float32)
    out = {}
    with fs.Graph(rp, ci, w) as g:
        for name, v in VARIANTS.items():
            for rates in (False, True):
                sim = fs.Sim.from_model(g, model, variant=v, record_rates=rates, replicas=2)
                sim.set_state(st, age, 0, step_index=5)
                sim.set_state(st, age, 1, step_index=5)
                sim.step(3)
                out[(name, rates)] = ([sim.get_state(r)[:2] for r in range(2)],
                                      sim.rates(0) if rates else None)
                sim.close()
    ref = out[("stream", True)]
    for key, (states, r0) in out.items():
        for (s0, a0), (s1, a1) in zip(ref[0], states):
            np.testing.assert_array_equal(s0, s1, err_msg=str(key))
            np.testing.assert_array_equal(a0, a1, err_msg=str(key))
        if r0 is not None:
            np.testing.assert_array_equal(ref[1], r0, err_msg=str(key))
