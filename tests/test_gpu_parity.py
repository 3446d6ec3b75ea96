"""Parity of the HIP step (through the C ABI) with the FP64 oracle.

Inputs are the seeded synthetic graphs of workloads/: the random 10-regular
graph with N = 1e4 (log-normal E and I, beta = 0.06, dt = 0.1, ten exposed
seeds) is the small case the oracle finishes in seconds; other sizes cover
ragged tails, replicas and the other holding-time laws.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W
from _parity import check_mismatch_budget, check_one_step, check_rates, guard_band_mismatches

pytestmark = pytest.mark.gpu

SMALL = W.WORKLOADS["regular10_n1e4"]


@pytest.fixture(scope="module")
def small_graph():
    rp, ci = W.workload_graph(SMALL["graph"])
    g = fs.Graph(rp, ci)
    yield rp, ci, g
    g.close()


def storage_of(compact):
    return fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32


def zero_age(n, compact):
    return np.zeros(n, np.uint16 if compact else np.float32)


# ------------------------------------------------------------ building blocks

def test_device_philox_matches_oracle():
    rng = np.random.default_rng(5)
    n = 1_000_000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    for seed in [0, 0x0123456789ABCDEF]:
        key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
        np.testing.assert_array_equal(fs.fs_eval_philox(ctr, seed), oracle.philox4x32(ctr, key))


HAZARD_LAWS = [
    W.LN_E, W.LN_I, ("lognormal", math.log(4.0), 0.668), ("lognormal", math.log(2.0), 0.3),
    ("lognormal", math.log(6.0), 0.8), ("weibull", 2.0, 6.0), ("weibull", 1.5, 3.0),
    ("weibull", 3.0, 8.0), ("weibull", 1.0, 4.0), ("erlang", 3, 1.0), ("erlang", 2, 1.0 / 3.0),
    ("erlang", 5, 5.0 / 6.0), ("erlang", 1, 0.5), ("exp", 0.25),
]


@pytest.mark.parametrize("law", HAZARD_LAWS, ids=lambda l: "-".join(str(x)[:6] for x in l))
def test_device_hazard_fp32_days_within_2e6(law):
    # float32 ages: every multiple-of-dt age the FP32 path accumulates over 400
    # days for dt = 0.1 and 0.2, plus a dense log grid
    ages = [np.zeros(1, np.float32)]
    for dt in [np.float32(0.1), np.float32(0.2)]:
        a = np.cumsum(np.full(4000, dt, np.float32), dtype=np.float32)
        ages.append(a)
    ages.append(np.geomspace(1e-3, 1e3, 200_000).astype(np.float32))
    tau = np.concatenate(ages)
    got = fs.fs_eval_hazard(law, tau, fs.FS_STORAGE_FP32)
    ref = oracle.hazard(law, tau.astype(np.float64))
    worst = check_rates(got, ref, f"hazard {law}")
    print(f"hazard {law}: max rel err {worst:.3e}")


@pytest.mark.parametrize("law", HAZARD_LAWS, ids=lambda l: "-".join(str(x)[:6] for x in l))
@pytest.mark.parametrize("dt", [0.1, 0.2])
def test_device_hazard_compact_steps_within_2e6(law, dt):
    n = np.arange(65536, dtype=np.uint16)
    got = fs.fs_eval_hazard(law, n, fs.FS_STORAGE_COMPACT, dt)
    ref = oracle.hazard(law, n.astype(np.float64) * dt)
    check_rates(got, ref, f"hazard {law} steps dt={dt}")


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
@pytest.mark.parametrize("laws", [(W.LN_E, W.LN_I), (("erlang", 3, 1.0), ("weibull", 2.0, 6.0))],
                         ids=["lognormal", "erlang-weibull"])
def test_hazard_table_serves_the_evaluated_hazards(small_graph, laws, compact):
    """Fixed-step sims take the hazard of an E/I unit whose age is one that
    fixed steps reach from 0 (a_m, m below the table length) from a table;
    the rates the step records must be exactly the directly evaluated
    hazards, for table ages, ages next to them and ages past the table."""
    rp, ci, g = small_graph
    n = len(rp) - 1
    dt = 0.1
    rng = np.random.default_rng(11)
    st = np.where(rng.random(n) < 0.5, fs.FS_E, fs.FS_I).astype(np.int32)
    m = rng.integers(0, 9000, n)                      # 8192 entries: some ages lie past the table
    if compact:
        age = m.astype(np.uint16)
    else:
        a = np.concatenate([[0], np.cumsum(np.full(9000, dt, np.float32), dtype=np.float32)]).astype(np.float32)
        age = a[m]
        off = rng.random(n) < 0.3                     # ages next to a table age: evaluated
        age[off] = np.nextafter(age[off], np.float32(np.inf))
    model = {"ei": laws[0], "ir": laws[1], "beta": 0.06, "dt": dt, "seed": 1}
    sim = fs.Sim.from_model(g, model, storage=storage_of(compact), record_rates=True)
    try:
        sim.set_state(st, age, 0, step_index=0)
        sim.step(1)
        got = sim.rates(0)
    finally:
        sim.close()
    storage = storage_of(compact)
    for comp, law in [(fs.FS_E, laws[0]), (fs.FS_I, laws[1])]:
        sel = st == comp
        want = fs.fs_eval_hazard(law, age[sel], storage, dt)
        np.testing.assert_array_equal(got[sel], want)


# ----------------------------------------------------------- one-step parity

def oracle_checkpoints(rp, ci, model, seeds, ks, compact):
    n = len(rp) - 1
    st = W.initial_state(n, seeds)
    age = zero_age(n, compact)
    out = {}
    k0 = 0
    for k in ks:
        if k > k0:
            st, age, _ = oracle.run((rp, ci), model, st, age, k - k0, step0=k0, compact=compact)
            k0 = k
        out[k] = (st.copy(), age.copy())
    return out


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
def test_one_step_parity_at_checkpoints(small_graph, compact):
    rp, ci, g = small_graph
    n = len(rp) - 1
    ks = [0, 50, 100, 150, 200, 250]
    total_upd, total_mism = 0, 0
    for seed in [0, 1, 2**40 + 3]:
        model = dict(SMALL["model"], seed=seed)
        seeds = W.seed_nodes(n, SMALL["seeds"], SMALL["seed_rng"] + seed % 7)
        cps = oracle_checkpoints(rp, ci, model, seeds, ks, compact)
        sim = fs.Sim.from_model(g, model, storage=storage_of(compact), record_rates=True)
        try:
            for k in ks:
                st, age = cps[k]
                sim.set_state(st, age, 0, step_index=k)
                sim.step(1)
                gst, gage, gk = sim.get_state(0)
                assert gk == k + 1
                ora = oracle.step((rp, ci), model, st, age, (st == 2).astype(np.float64), k,
                                  compact=compact)
                label = f"seed={seed} k={k} {'compact' if compact else 'fp32'}"
                nm, worst = check_one_step({"state": gst, "age": gage, "rates": sim.rates(0)},
                                           ora, st, label)
                total_upd += n
                total_mism += nm
                # per-step counts recorded by the kernel equal an exact recount
                np.testing.assert_array_equal(sim.history(k, 1)[0], np.bincount(gst, minlength=4))
                np.testing.assert_array_equal(sim.counts(0), np.bincount(gst, minlength=4))
        finally:
            sim.close()
    check_mismatch_budget(total_mism, total_upd, "checkpoints")


# ------------------------------------------------------- whole trajectories

VARIANTS = {"stream": fs.VARIANT_STREAM, "resident": fs.VARIANT_RESIDENT,
            "summary": fs.VARIANT_SUMMARY}


def run_gpu(g, model, seeds, steps, n, compact=False, b=0, replicas=1, variant=0):
    sim = fs.Sim.from_model(g, model, storage=storage_of(compact), steps_per_graph=b,
                            replicas=replicas, variant=variant)
    sim.seed(seeds, replica=-1, compartment=fs.FS_E)
    sim.step(steps)
    res = [(*sim.get_state(r)[:2], sim.history(0, steps, r)) for r in range(replicas)]
    sim.close()
    return res


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
def test_trajectory_matches_oracle(small_graph, compact, variant):
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = SMALL["model"]
    seeds = W.seed_nodes(n, SMALL["seeds"], SMALL["seed_rng"])
    steps = SMALL["steps"]
    (gst, gage, ghist), = run_gpu(g, model, seeds, steps, n, compact, b=50,
                                  variant=VARIANTS[variant])
    ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), zero_age(n, compact),
                                  steps, compact=compact)
    # a divergence would have to start at a guard-band draw; none is expected
    # (about 1e-3 over the whole run), so the trajectories are compared exactly
    np.testing.assert_array_equal(ghist, ohist)
    np.testing.assert_array_equal(gst, ost)
    np.testing.assert_array_equal(gage, oage)
    np.testing.assert_array_equal(ghist.sum(1), n)


def test_graph_replay_equals_eager(small_graph):
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.15)
    seeds = W.seed_nodes(n, 40, 3)
    ref = run_gpu(g, model, seeds, 137, n, b=0)[0]
    for b in [50, 7, 1]:
        got = run_gpu(g, model, seeds, 137, n, b=b)[0]
        for x, y in zip(got, ref):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
def test_all_variants_identical(compact):
    # a scale-free graph (hub rows take the degree-binned path)
    n = 20_000
    rp, ci = W.barabasi_albert(n, 4, 6)
    model = {"ei": ("erlang", 3, 1.0), "ir": ("weibull", 2.0, 6.0), "beta": 0.08, "dt": 0.1,
             "seed": 21}
    seeds = W.seed_nodes(n, 30, 1)
    with fs.Graph(rp, ci) as g:
        runs = {name: run_gpu(g, model, seeds, 150, n, compact, b=25, replicas=2, variant=v)
                for name, v in VARIANTS.items()}
    for name in ["resident", "summary"]:
        for ra, rb in zip(runs["stream"], runs[name]):
            for x, y in zip(ra, rb):
                np.testing.assert_array_equal(x, y)


def test_all_variants_identical_weighted_hubs():
    # float pressures: the heavy-row kernels of the resident and the other
    # variants sum each lane's edges in one order and fold them by one tree,
    # so weighted trajectories agree bit for bit too
    n = 20_000
    rp, ci = W.barabasi_albert(n, 5, 12)
    w = np.random.default_rng(3).uniform(0.2, 1.8, len(ci)).astype(np.float32)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.08, "dt": 0.1, "seed": 4}
    seeds = W.seed_nodes(n, 30, 2)
    with fs.Graph(rp, ci, w) as g:
        runs = {}
        for name, v in VARIANTS.items():
            sim = fs.Sim.from_model(g, model, steps_per_graph=25, variant=v, heavy_degree=16, segment_edges=64)
            assert sim.bins()[2] > 1000
            sim.seed(seeds, replica=-1, compartment=fs.FS_E)
            sim.step(150)
            runs[name] = (*sim.get_state(0)[:2], sim.history(0, 150, 0))
            sim.close()
    for name in ["resident", "summary"]:
        for x, y in zip(runs["stream"], runs[name]):
            np.testing.assert_array_equal(x, y)
    assert runs["stream"][2][-1, 1:].sum() > 300   # the epidemic grew from its 30 seeds


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_long_push_list_of_a_hub(variant):
    """A center joined to 1200 sub-hubs of 20 leaves each: with bins (12, 512)
    the center and the sub-hubs are binned rows, and the center's own push
    list (the 1200 sub-hubs) is longer than 64 entries, so its changes of
    state are pushed in rounds of coalesced list loads (three rounds of 512).
    The trajectory, seeded at the center, matches the oracle."""
    hubs, leaves = 1200, 20
    n = 1 + hubs + hubs * leaves
    sub = np.arange(1, hubs + 1)
    src = np.concatenate([np.zeros(hubs, np.int64), np.repeat(sub, leaves)])
    dst = np.concatenate([sub, np.arange(hubs + 1, n)])
    rp, ci = W.csr_from_edges(n, src, dst)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 9}
    seeds = np.array([0], np.int64)
    steps = 200
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, model, steps_per_graph=25, variant=VARIANTS[variant], heavy_degree=12,
                                segment_edges=512)
        sim.seed(seeds, replica=-1, compartment=fs.FS_E)
        sim.step(steps)
        gst, gage = sim.get_state(0)[:2]
        ghist = sim.history(0, steps, 0)
        sim.close()
    ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), zero_age(n, False), steps)
    np.testing.assert_array_equal(ghist, ohist)
    np.testing.assert_array_equal(gst, ost)
    np.testing.assert_array_equal(gage, oage)
    assert ost[0] == fs.FS_R and ohist[-1][3] > hubs  # the center recovered after infecting sub-hubs


def test_summary_variant_with_coarse_groups():
    """N*R just above 2^26 units makes each summary bit cover 128 units (two
    bitmap words).  Contacts form a random 8-regular graph on 200k nodes spread
    over the whole id range; every other node is isolated.  The summary and
    streaming variants agree exactly and one step matches the oracle."""
    n, R = (1 << 25) + 1000, 2
    rng = np.random.default_rng(11)
    sub = np.sort(rng.choice(n, 200_000, replace=False))
    srp, sci = W.random_regular_matchings(len(sub), 8, 4)
    deg = np.zeros(n, np.int64)
    deg[sub] = 8
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=rp[1:])
    rp = rp.astype(np.int32)
    ci = sub[sci].astype(np.int32)  # rows of sub[i] keep their order
    model = dict(SMALL["model"], beta=0.2, seed=5)
    seeds = sub[rng.choice(len(sub), 300, replace=False)]
    with fs.Graph(rp, ci) as g:
        out = {}
        for name in ["summary", "stream"]:
            sim = fs.Sim.from_model(g, model, steps_per_graph=20, replicas=R, variant=VARIANTS[name],
                                    record_rates=True)
            sim.seed(seeds, replica=-1, compartment=fs.FS_E)
            sim.step(80)
            st, age, k = sim.get_state(1)
            sim.step(1)
            out[name] = (st, age, *sim.get_state(1)[:2], sim.history(0, 81, 1), sim.rates(1))
            sim.close()
    for x, y in zip(out["summary"], out["stream"]):
        np.testing.assert_array_equal(x, y)
    st, age, gst, gage, hist, rates = out["summary"]
    assert hist[-2, 2] > 50  # infection spread along the contacts
    nodes = np.concatenate([sub[rng.choice(len(sub), 50_000, replace=False)],
                            rng.choice(n, 10_000, replace=False)])
    ora = oracle.step_nodes((rp, ci), model, st, age, (st == 2).astype(np.float64), 80, nodes,
                            replica=1)
    nm = guard_band_mismatches(gst[nodes], ora["state"], ora["u"], ora["q"], "coarse summary")
    check_mismatch_budget(nm, len(nodes), "coarse summary")
    check_rates(rates[nodes], ora["lam"], "coarse summary")


def test_resident_variant_size_limit():
    # the LDS-resident bitmap holds at most 2^20 units; larger sims take the
    # summary variant automatically and refuse an explicit resident request
    n = (1 << 20) + 1
    rp = np.zeros(n + 1, np.int32)
    with fs.Graph(rp, np.zeros(0, np.int32)) as g:
        with pytest.raises(fs.FsError):
            fs.Sim(g, W.LN_E, W.LN_I, 0.1, 0.1, variant=fs.VARIANT_RESIDENT)
        sim = fs.Sim(g, W.LN_E, W.LN_I, 0.1, 0.1, variant=fs.VARIANT_AUTO)
        sim.seed([0, n - 1], replica=0, compartment=fs.FS_I)
        sim.step(3)
        assert sim.counts(0)[2] + sim.counts(0)[3] == 2
        sim.close()


def test_split_step_calls_equal_one_call(small_graph):
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = SMALL["model"]
    seeds = W.seed_nodes(n, 10, 9)
    sim = fs.Sim.from_model(g, model, steps_per_graph=10)
    sim.seed(seeds, replica=0)
    for chunk in [3, 10, 25, 1, 61]:
        sim.step(chunk)
    a = sim.get_state(0)
    ha = sim.history(0, 100)
    sim.close()
    (st, age, hist), = run_gpu(g, model, seeds, 100, n, b=0)
    np.testing.assert_array_equal(a[0], st)
    np.testing.assert_array_equal(a[1], age)
    np.testing.assert_array_equal(ha, hist)


def test_checkpoint_resume_is_bit_exact(small_graph):
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.12, seed=77)
    seeds = W.seed_nodes(n, 25, 4)
    sim = fs.Sim.from_model(g, model, steps_per_graph=20)
    sim.seed(seeds, replica=0)
    sim.step(120)
    st, age, k = sim.get_state(0)
    sim.step(80)
    final = sim.get_state(0)
    h_tail = sim.history(120, 80)
    sim.close()
    sim2 = fs.Sim.from_model(g, model, steps_per_graph=20)
    sim2.set_state(st, age, 0, step_index=k)
    sim2.step(80)
    resumed = sim2.get_state(0)
    np.testing.assert_array_equal(sim2.history(120, 80), h_tail)
    sim2.close()
    np.testing.assert_array_equal(resumed[0], final[0])
    np.testing.assert_array_equal(resumed[1], final[1])
    assert resumed[2] == final[2] == 200


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_sixteen_replicas_on_a_degree_sorted_graph(variant, compact):
    # 16 replicas of a unit-weight graph run the instantiations that know the
    # replica count; on a BA graph (degree-sorted, mixed layout with binned
    # rows) every variant must still give each replica the oracle's trajectory
    n = 3000
    rp, ci = W.barabasi_albert(n, 3, 17)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.12, "dt": 0.1, "seed": 23}
    seeds = W.seed_nodes(n, 20, 4)
    steps = 120
    with fs.Graph(rp, ci) as g:
        res = run_gpu(g, model, seeds, steps, n, compact, b=30, replicas=16, variant=VARIANTS[variant])
    for r in [0, 7, 15]:
        ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), zero_age(n, compact), steps,
                                      replica=r, compact=compact)
        np.testing.assert_array_equal(res[r][2], ohist, err_msg=f"replica {r}")
        np.testing.assert_array_equal(res[r][0], ost)
        np.testing.assert_array_equal(res[r][1], oage)
    assert ohist[-1][0] < n - 100  # the epidemic spread


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("replicas", [4, 16, 64])
def test_replicas_match_oracle_per_replica(replicas, variant):
    n = 1500  # not a multiple of the workgroup size
    rp, ci = W.random_regular(n, 10, 11)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.15, "dt": 0.1, "seed": 5}
    seeds = W.seed_nodes(n, 15, 2)
    steps = 120
    with fs.Graph(rp, ci) as g:
        res = run_gpu(g, model, seeds, steps, n, b=30, replicas=replicas,
                      variant=VARIANTS[variant])
    check = range(replicas) if replicas <= 16 else [0, 1, 31, 63]
    for r in check:
        ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds),
                                      np.zeros(n, np.float32), steps, replica=r)
        np.testing.assert_array_equal(res[r][2], ohist, err_msg=f"replica {r}")
        np.testing.assert_array_equal(res[r][0], ost)
        np.testing.assert_array_equal(res[r][1], oage)


def test_other_laws_on_scale_free_graph():
    # Erlang(k=3, mean 3 d) and Weibull(2, 6 d) on a small Barabasi-Albert graph
    n = 5000
    rp, ci = W.barabasi_albert(n, 5, 2)
    model = W.WORKLOADS["ba5_n1e6"]["model"]
    seeds = W.seed_nodes(n, 20, 8)
    for compact in [False, True]:
        with fs.Graph(rp, ci) as g:
            (gst, gage, ghist), = run_gpu(g, model, seeds, 200, n, compact, b=25)
        ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds),
                                      zero_age(n, compact), 200, compact=compact)
        np.testing.assert_array_equal(ghist, ohist)
        np.testing.assert_array_equal(gst, ost)
        np.testing.assert_array_equal(gage, oage)


def test_weighted_graph_one_step():
    n = 3000
    rp, ci = W.random_regular(n, 8, 12)
    w = np.random.default_rng(1).random(len(ci)).astype(np.float32) * 2
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 3}
    rng = np.random.default_rng(4)
    st = rng.choice(4, size=n, p=[0.6, 0.1, 0.2, 0.1]).astype(np.int32)
    age = (rng.integers(0, 200, n) * np.float32(0.1)).astype(np.float32)
    with fs.Graph(rp, ci, w) as g:
        sim = fs.Sim.from_model(g, model, record_rates=True)
        sim.set_state(st, age, 0, step_index=42)
        sim.step(1)
        gst, gage, _ = sim.get_state(0)
        rates = sim.rates(0)
        sim.close()
    ora = oracle.step((rp, ci, w), model, st, age, (st == 2).astype(np.float64), 42)
    # weighted pressures are sums of float32 products: rounding order differs
    # from the oracle's FP64 sum, so rates agree to ~d ulps rather than exactly
    check_one_step({"state": gst, "age": gage, "rates": rates}, ora, st, "weighted")


# ------------------------------------------------------------- packed columns

PACKED_CASES = [
    # (n, degree, variant, compact): 20-bit columns up to 2^20 nodes, 24-bit
    # above; ragged last chunks; degrees below and at the preload depths
    (50_000, 10, fs.VARIANT_RESIDENT, False),
    (50_004, 7, fs.VARIANT_RESIDENT, True),
    (50_000, 10, fs.VARIANT_SUMMARY, True),
    (50_000, 12, fs.VARIANT_STREAM, False),
    (1_100_000, 8, fs.VARIANT_SUMMARY, True),
    (1_100_002, 9, fs.VARIANT_STREAM, False),
]


@pytest.mark.parametrize("n,d,variant,compact", PACKED_CASES,
                         ids=[f"n{c[0]}-d{c[1]}-v{c[2]}-{'compact' if c[3] else 'fp32'}" for c in PACKED_CASES])
def test_packed_columns_match_plain_and_oracle(n, d, variant, compact):
    # packed columns (the step's transposed copy of the graph with 20 or 24
    # bits per column) give the trajectory of 32-bit columns bit for bit;
    # the small graphs match the oracle's whole trajectory, the large ones
    # its next step on a sample of nodes
    rp, ci = W.random_regular(n, d, 5)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.08, "dt": 0.1, "seed": 21}
    seeds = W.seed_nodes(n, 60, 4)
    steps = 120
    storage = storage_of(compact)
    out = {}
    with fs.Graph(rp, ci) as g:
        for cols in (fs.FS_COLUMNS_AUTO, fs.FS_COLUMNS_PLAIN):
            with fs.Sim.from_model(g, model, variant=variant, storage=storage, steps_per_graph=20,
                                   history_len=steps, columns=cols) as sim:
                out[cols] = sim.column_bits()
                sim.seed(seeds, replica=0)
                sim.step(steps)
                out[cols, "state"] = sim.get_state(0)
                out[cols, "hist"] = sim.history(0, steps)
                if cols == fs.FS_COLUMNS_AUTO:
                    sim.step(1)
                    out["next"] = sim.get_state(0)
    assert out[fs.FS_COLUMNS_AUTO] == (20 if n <= 1 << 20 else 24)
    assert out[fs.FS_COLUMNS_PLAIN] == 32
    np.testing.assert_array_equal(out[fs.FS_COLUMNS_AUTO, "hist"], out[fs.FS_COLUMNS_PLAIN, "hist"])
    for a, b in zip(out[fs.FS_COLUMNS_AUTO, "state"], out[fs.FS_COLUMNS_PLAIN, "state"]):
        np.testing.assert_array_equal(a, b)
    st, age, k = out[fs.FS_COLUMNS_AUTO, "state"]
    assert (st != 0).sum() > 100  # the epidemic is under way
    if n <= 100_000:
        ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), zero_age(n, compact), steps,
                                      compact=compact)
        np.testing.assert_array_equal(out[fs.FS_COLUMNS_AUTO, "hist"], ohist)
        np.testing.assert_array_equal(st, ost)
        np.testing.assert_array_equal(age, oage)
    else:
        gst, gage, _ = out["next"]
        nodes = np.unique(np.concatenate([np.random.default_rng(1).choice(n, 30_000, replace=False),
                                          np.flatnonzero(st != 0)[:30_000]]))
        ora = oracle.step_nodes((rp, ci), model, st, age, (st == 2).astype(np.float64), k, nodes,
                                compact=compact)
        nm = guard_band_mismatches(gst[nodes], ora["state"], ora["u"], ora["q"], "packed sample")
        check_mismatch_budget(nm, len(nodes), "packed sample")
        same = gst[nodes] == ora["state"]
        np.testing.assert_array_equal(gage[nodes][same], ora["age"][same])


BA_PACKED_CASES = [
    # (variant, heavy_degree, segment_edges, compact): degree-sorted graphs
    # pack the chunks whose rows share one degree of at most 12; binned rows
    # (pushed pressure), deeper uniform chunks and mixed chunks keep 32 bits
    (fs.VARIANT_RESIDENT, 0, 0, False),
    (fs.VARIANT_RESIDENT, 12, 512, True),
    (fs.VARIANT_SUMMARY, 32, 256, False),
    (fs.VARIANT_STREAM, -1, 0, False),
]


@pytest.mark.parametrize("variant,hd,se,compact", BA_PACKED_CASES,
                         ids=[f"v{c[0]}-bins{c[1]}-{c[2]}-{'compact' if c[3] else 'fp32'}" for c in BA_PACKED_CASES])
def test_packed_columns_degree_sorted_graph(variant, hd, se, compact):
    n = 30_000
    rp, ci = W.barabasi_albert(n, 4, 8)
    model = {"ei": ("erlang", 3, 1.0), "ir": ("weibull", 2.0, 6.0), "beta": 0.05, "dt": 0.1, "seed": 17}
    seeds = W.seed_nodes(n, 30, 3)
    steps = 150
    storage = storage_of(compact)
    out = {}
    with fs.Graph(rp, ci) as g:
        for cols in (fs.FS_COLUMNS_AUTO, fs.FS_COLUMNS_PLAIN):
            with fs.Sim.from_model(g, model, variant=variant, storage=storage, steps_per_graph=25,
                                   history_len=steps, heavy_degree=hd, segment_edges=se, columns=cols) as sim:
                out[cols] = sim.column_bits()
                sim.seed(seeds, replica=0)
                sim.step(steps)
                out[cols, "state"] = sim.get_state(0)
                out[cols, "hist"] = sim.history(0, steps)
    assert out[fs.FS_COLUMNS_AUTO] == 20 and out[fs.FS_COLUMNS_PLAIN] == 32
    np.testing.assert_array_equal(out[fs.FS_COLUMNS_AUTO, "hist"], out[fs.FS_COLUMNS_PLAIN, "hist"])
    for a, b in zip(out[fs.FS_COLUMNS_AUTO, "state"], out[fs.FS_COLUMNS_PLAIN, "state"]):
        np.testing.assert_array_equal(a, b)
    ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), zero_age(n, compact), steps,
                                  compact=compact)
    np.testing.assert_array_equal(out[fs.FS_COLUMNS_AUTO, "hist"], ohist)
    st, age, _ = out[fs.FS_COLUMNS_AUTO, "state"]
    np.testing.assert_array_equal(st, ost)
    np.testing.assert_array_equal(age, oage)
    assert ohist[-1, 0] < n - 1000  # the epidemic spread


def test_column_bits_follow_the_rules():
    rp, ci = W.random_regular(3000, 6, 1)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.1, "dt": 0.1, "seed": 1}
    w = np.full(len(ci), 0.5, np.float32)
    brp, bci = W.barabasi_albert(3000, 3, 2)
    with fs.Graph(rp, ci) as g, fs.Graph(rp, ci, w) as gw, fs.Graph(brp, bci) as gb:
        for graph, kw, bits in [
            (g, {}, 20), (g, {"variant": fs.VARIANT_STREAM}, 20), (g, {"variant": fs.VARIANT_SUMMARY}, 20),
            (g, {"storage": fs.FS_STORAGE_COMPACT}, 20), (g, {"adaptive": True}, 20),
            (g, {"replicas": 4}, 32), (g, {"record_rates": True}, 20), (g, {"compaction": True}, 20),
            (g, {"columns": fs.FS_COLUMNS_PLAIN}, 32), (g, {"shed": ("density", W.LN_I, 1.0)}, 20),
            (g, {"shed": ("density", W.LN_I, 1.0), "record_rates": True}, 32),
            (g, {"shed": ("density", W.LN_I, 1.0), "compaction": True}, 32),
            (gw, {}, 32), (gb, {}, 20), (gb, {"replicas": 2}, 32),
        ]:
            with fs.Sim.from_model(graph, model, **kw) as sim:
                assert sim.column_bits() == bits, kw
        with pytest.raises(fs.FsError):
            fs.Sim.from_model(g, model, columns=2)


# ------------------------------------------------------------- edge cases

@pytest.mark.gpu
@pytest.mark.parametrize("deg", [4, 6, 9, 11])
def test_uniform_degree_below_preload_depth(deg):
    # uniform graphs whose degree is below the kernel's preload depth (8, 10
    # or 12 slots): the slots past the degree read no column and must not
    # count node 0's bit, which is set here (Eq. (influence) sums over the
    # row only); every variant, with and without rate recording, and a
    # replicated sim
    n = 2000
    rp, ci = W.random_regular(n, deg, 5)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.3, "dt": 0.1, "seed": 11}
    rng = np.random.default_rng(deg)
    st = np.where(rng.random(n) < 0.9, 0, rng.integers(1, 4, n)).astype(np.int32)
    st[0] = 2
    age = (rng.integers(0, 50, n) * np.float32(0.1)).astype(np.float32)
    iota = (st == 2).astype(np.float64)
    with fs.Graph(rp, ci) as g:
        for variant in (fs.VARIANT_RESIDENT, fs.VARIANT_SUMMARY, fs.VARIANT_STREAM):
            for rates in (True, False):
                for R in (1, 4):
                    sim = fs.Sim.from_model(g, model, variant=variant, record_rates=rates, replicas=R)
                    for r in range(R):
                        sim.set_state(st, age, r, step_index=5)
                    sim.step(1)
                    for r in range(R):
                        gst, gage, _ = sim.get_state(r)
                        ora = oracle.step((rp, ci), model, st, age, iota, 5, replica=r)
                        check_one_step({"state": gst, "age": gage, "rates": sim.rates(r) if rates else None},
                                       ora, st, f"degree {deg} variant {variant} rates {rates} R {R} r {r}")
                    sim.close()



def test_edge_cases_tiny_graphs():
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.5, "dt": 0.1, "seed": 1}
    cases = {
        "single isolated node": (np.array([0, 0]), np.zeros(0)),
        "single self-loop": (np.array([0, 1]), np.array([0])),
        "empty rows and a multi-edge": (np.array([0, 0, 3, 3, 4]), np.array([0, 0, 3, 1])),
        "ragged 257": W.random_regular(257, 4, 1),
    }
    for name, (rp, ci) in cases.items():
        n = len(rp) - 1
        rng = np.random.default_rng(n)
        st = rng.integers(0, 4, n).astype(np.int32)
        age = (rng.integers(0, 100, n) * np.float32(0.1)).astype(np.float32)
        with fs.Graph(rp, ci) as g:
            sim = fs.Sim.from_model(g, model, record_rates=True)
            sim.set_state(st, age, 0, step_index=3)
            sim.step(1)
            gst, gage, _ = sim.get_state(0)
            rates = sim.rates(0)
            np.testing.assert_array_equal(sim.counts(0), np.bincount(gst, minlength=4))
            sim.close()
        ora = oracle.step((rp, ci), model, st, age, (st == 2).astype(np.float64), 3)
        check_one_step({"state": gst, "age": gage, "rates": rates}, ora, st, name)


def test_all_recovered_is_a_fixed_point():
    n = 1000
    rp, ci = W.random_regular(n, 6, 3)
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim(g, W.LN_E, W.LN_I, 0.5, 0.1, steps_per_graph=5)
        sim.set_state(np.full(n, 3, np.int32), np.zeros(n, np.float32), 0, step_index=0)
        sim.step(12)
        st, age, _ = sim.get_state(0)
        hist = sim.history(0, 12)
        sim.close()
    assert np.all(st == 3)
    np.testing.assert_array_equal(hist, np.tile([0, 0, 0, n], (12, 1)))
    a = np.float32(0.0)
    for _ in range(12):
        a = np.float32(a + np.float32(0.1))
    np.testing.assert_array_equal(age, a)  # ages of R nodes still advance (never used)


def test_history_window_and_errors(small_graph):
    rp, ci, g = small_graph
    sim = fs.Sim.from_model(g, SMALL["model"], history_len=8)
    try:
        sim.seed([1, 2, 3], replica=0)
        sim.step(20)
        h = sim.history(12, 8)  # the last history_len steps are kept
        st, _, _ = sim.get_state(0)
        np.testing.assert_array_equal(h[-1], np.bincount(st, minlength=4))
        with pytest.raises(fs.FsError):
            sim.history(11, 2)
        with pytest.raises(fs.FsError):
            sim.history(15, 6)
        with pytest.raises(fs.FsError):
            fs.fs_graph_destroy(g.handle)  # still used by the sim
    finally:
        sim.close()


# ----------------------------------------------- full size, sampled parity

def test_full_size_regular10_n1e6_sampled_parity():
    wl = W.WORKLOADS["regular10_n1e6"]
    rp, ci = W.workload_graph(wl["graph"])
    n = len(rp) - 1
    model = wl["model"]
    seeds = W.seed_nodes(n, wl["seeds"], wl["seed_rng"])
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, model, steps_per_graph=50, record_rates=True, columns=fs.FS_COLUMNS_PLAIN)
        sim.seed(seeds, replica=0)
        sim.step(400)  # the launch configuration of the benchmark: captured b = 50 steps
        st, age, k = sim.get_state(0)
        hist = sim.history(0, 400)
        np.testing.assert_array_equal(hist[-1], np.bincount(st, minlength=4))
        np.testing.assert_array_equal(hist.sum(1), n)
        sim.step(1)
        gst, gage, _ = sim.get_state(0)
        rates = sim.rates(0)
        sim.close()
        # the benchmark's own launch (no rate recording) runs the step with
        # 20-bit packed columns: the same trajectory, bit for bit
        with fs.Sim.from_model(g, model, steps_per_graph=50) as packed:
            assert packed.column_bits() == 20
            packed.seed(seeds, replica=0)
            packed.step(401)
            pst, page, _ = packed.get_state(0)
            np.testing.assert_array_equal(packed.history(0, 400), hist)
            np.testing.assert_array_equal(pst, gst)
            np.testing.assert_array_equal(page, gage)
    nodes = np.random.default_rng(0).choice(n, 100_000, replace=False)
    iota = (st == 2).astype(np.float64)
    ora = oracle.step_nodes((rp, ci), model, st, age, iota, k, nodes)
    nm = guard_band_mismatches(gst[nodes], ora["state"], ora["u"], ora["q"], "N=1e6 sample")
    check_mismatch_budget(nm, len(nodes), "N=1e6 sample")
    same = gst[nodes] == ora["state"]
    np.testing.assert_array_equal(gage[nodes][same], ora["age"][same])
    check_rates(rates[nodes], ora["lam"], "N=1e6 sample")
    assert (st != 0).sum() > 1000  # the epidemic is under way at the checkpoint


def test_full_size_ba5_n1e6_sampled_parity():
    # the Barabasi-Albert workload at its full size in the benchmark's launch
    # configuration: explicit degree bins (32, 256) (heavy rows of up to ~4200
    # edges in segments of 256, i.e. up to 17 segments each), the resident
    # variant, captured b = 50 steps; one step from steps 250 and 350 (the
    # epidemic under way) compared node by node on every heavy row and
    # 100000 others
    wl = W.WORKLOADS["ba5_n1e6"]
    rp, ci = W.workload_graph(wl["graph"])
    n = len(rp) - 1
    model = wl["model"]
    seeds = W.seed_nodes(n, wl["seeds"], wl["seed_rng"])
    deg = np.diff(rp)
    heavy = np.flatnonzero(deg > 32)
    rest = np.setdiff1d(np.random.default_rng(1).choice(n, 100_000, replace=False), heavy)
    nodes = np.concatenate([heavy, rest])
    multi = 0
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, model, steps_per_graph=50, record_rates=True,
                                heavy_degree=32, segment_edges=256)
        hd, se, nseg = sim.bins()
        assert (hd, se) == (32, 256) and nseg >= len(heavy)
        sim.seed(seeds, replica=0)
        done = 0
        for k0 in (250, 350):
            sim.step(k0 - done)
            st, age, k = sim.get_state(0)
            assert k == k0
            hist = sim.history(k0 - 50, 50)
            np.testing.assert_array_equal(hist[-1], np.bincount(st, minlength=4))
            sim.step(1)
            done = k0 + 1
            gst, gage, _ = sim.get_state(0)
            rates = sim.rates(0)
            iota = (st == 2).astype(np.float64)
            ora = oracle.step_nodes((rp, ci), model, st, age, iota, k, nodes)
            label = f"BA N=1e6 sample, step {k}"
            nm = guard_band_mismatches(gst[nodes], ora["state"], ora["u"], ora["q"], label)
            check_mismatch_budget(nm, len(nodes), label)
            same = gst[nodes] == ora["state"]
            np.testing.assert_array_equal(gage[nodes][same], ora["age"][same], err_msg=label)
            check_rates(rates[nodes], ora["lam"], label)
            # susceptible hub rows with infectious neighbours were exercised
            hub_s = heavy[(st[heavy] == 0) & (ora["lam"][:len(heavy)] > 0)]
            assert len(hub_s) > 1000, label
            multi += int((deg[hub_s] > 256).sum())
        sim.close()
    assert multi >= 5  # multi-segment rows among them
    assert (st != 0).sum() > 50_000


# ------------------------------------------------------ ensemble statistics

def test_ensemble_peak_prevalence_and_attack_rate(small_graph):
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.08, seed=1234)
    seeds = W.seed_nodes(n, SMALL["seeds"], SMALL["seed_rng"])
    steps, R = 300, 256   # four sims of 64 replicas (replica ids 0..63 of four seeds)
    res = []
    for j in range(R // 64):
        res += run_gpu(g, dict(model, seed=1234 + j), seeds, steps, n, b=50, replicas=64)
    gpk = np.array([h[:, 2].max() / n for _, _, h in res])
    gar = np.array([1 - h[-1, 0] / n for _, _, h in res])
    opk, oar = [], []
    for r in range(64, 64 + R):  # independent oracle replicas (other Philox streams)
        _, _, h = oracle.run((rp, ci), model, W.initial_state(n, seeds), np.zeros(n, np.float32),
                             steps, replica=r)
        opk.append(h[:, 2].max() / n)
        oar.append(1 - h[-1, 0] / n)
    opk, oar = np.array(opk), np.array(oar)
    for a, b, name in [(gpk, opk, "peak prevalence"), (gar, oar, "attack rate")]:
        se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
        assert abs(a.mean() - b.mean()) < 3 * se, (name, a.mean(), b.mean(), se)


# ------------------------------------------------------ degree-binned rows

@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("replicas", [1, 4])
def test_degree_bins_give_identical_results(variant, replicas):
    # Barabasi-Albert hubs: the same trajectory with no bins, with fine bins
    # (many multi-segment rows) and with the defaults; unit weights make the
    # pressures exact integers in any summation order
    n = 20_000
    rp, ci = W.barabasi_albert(n, 5, 9)
    model = W.WORKLOADS["ba5_n1e6"]["model"]
    seeds = W.seed_nodes(n, 40, 3)
    outs = []
    with fs.Graph(rp, ci) as g:
        for hd, se in [(-1, 0), (8, 64), (0, 0)]:
            sim = fs.Sim.from_model(g, model, steps_per_graph=20, replicas=replicas,
                                    variant=VARIANTS[variant], heavy_degree=hd, segment_edges=se)
            b = sim.bins()
            if hd == 8:
                assert b[2] > 1000  # segments
            sim.seed(seeds, replica=-1)
            sim.step(150)
            outs.append([(*sim.get_state(r)[:2], sim.history(0, 150, r)) for r in range(replicas)])
            sim.close()
    for other in outs[1:]:
        for ra, rb in zip(outs[0], other):
            for x, y in zip(ra, rb):
                np.testing.assert_array_equal(x, y)
    ost, oage, ohist = oracle.run((rp, ci), model, W.initial_state(n, seeds), np.zeros(n, np.float32),
                                  150, replica=0)
    np.testing.assert_array_equal(outs[0][0][2], ohist)


def test_degree_bins_weighted_one_step():
    n = 8000
    rp, ci = W.barabasi_albert(n, 4, 10)
    w = np.random.default_rng(2).random(len(ci)).astype(np.float32)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.05, "dt": 0.1, "seed": 8}
    rng = np.random.default_rng(5)
    st = rng.choice(4, size=n, p=[0.5, 0.1, 0.3, 0.1]).astype(np.int32)
    age = (rng.integers(0, 200, n) * np.float32(0.1)).astype(np.float32)
    with fs.Graph(rp, ci, w) as g:
        sim = fs.Sim.from_model(g, model, record_rates=True, heavy_degree=16, segment_edges=64)
        sim.set_state(st, age, 0, step_index=5)
        sim.step(1)
        gst, gage, _ = sim.get_state(0)
        rates = sim.rates(0)
        sim.close()
    ora = oracle.step((rp, ci, w), model, st, age, (st == 2).astype(np.float64), 5)
    check_one_step({"state": gst, "age": gage, "rates": rates}, ora, st, "weighted bins")


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("replicas", [1, 4])
def test_pushed_hub_pressure_equals_gathered(variant, replicas):
    # Binned rows of an unweighted graph keep their pressure up to date by
    # pushes from the units entering and leaving I; the same graph with every
    # weight 1.0 gathers it from segment partials every step.  Both are the
    # exact integer count of infectious in-neighbours, so the trajectories are
    # identical, through a mid-run state load, a change of bins and a graph
    # replay / eager mix, and equal the oracle's.
    n = 20_000
    rp, ci = W.barabasi_albert(n, 5, 13)
    model = W.WORKLOADS["ba5_n1e6"]["model"]
    seeds = W.seed_nodes(n, 40, 8)
    ones = np.ones(len(ci), np.float32)
    outs = []
    for w in (None, ones):
        with fs.Graph(rp, ci, w) as g:
            sim = fs.Sim.from_model(g, model, steps_per_graph=20, replicas=replicas,
                                    variant=VARIANTS[variant], heavy_degree=12, segment_edges=64)
            sim.seed(seeds, replica=-1)
            sim.step(47)
            # a state load of replica 0 at a later step index (the pushed counts
            # are rebuilt from the loaded bitmap)
            st, age, _ = sim.get_state(0)
            st = st.copy()
            st[np.arange(0, n, 97)] = fs.FS_I
            sim.set_state(st, age, 0, step_index=60)
            sim.step(33)
            sim.set_bins(24, 128)   # new bins mid-run
            sim.step(41)
            outs.append([(*sim.get_state(r)[:2], sim.history(60, 74, r)) for r in range(replicas)])
            sim.close()
    for ra, rb in zip(outs[0], outs[1]):
        for x, y in zip(ra, rb):
            np.testing.assert_array_equal(x, y)
    # replica 0 from the loaded state against the oracle
    ost, oage, ohist = oracle.run((rp, ci), model, st, age, 74, step0=60, replica=0)
    np.testing.assert_array_equal(outs[0][0][2], ohist)
    np.testing.assert_array_equal(outs[0][0][0], ost)


def test_tune_restores_state_and_keeps_results():
    n = 30_000
    rp, ci = W.barabasi_albert(n, 5, 4)
    model = W.WORKLOADS["ba5_n1e6"]["model"]
    seeds = W.seed_nodes(n, 50, 6)
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, model, steps_per_graph=10)
        sim.seed(seeds, replica=0)
        sim.step(30)
        before = sim.get_state(0)
        hd, se = sim.tune(5)
        after = sim.get_state(0)
        assert sim.bins()[:2] == (hd, se)
        for x, y in zip(before, after):
            np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(sim.history(0, 30)[-1], np.bincount(after[0], minlength=4))
        sim.step(40)
        tuned = sim.get_state(0)
        sim.close()
        ref = fs.Sim.from_model(g, model, heavy_degree=-1)
        ref.seed(seeds, replica=0)
        ref.step(70)
        plain = ref.get_state(0)
        ref.close()
    for x, y in zip(tuned, plain):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("replicas", [1, 4])
def test_autotune_variants_cache_and_results(tmp_path, replicas):
    # the autotuner times variants and bins from a mid-run state, restores
    # it, and the run continues exactly as an untuned one; the choice is
    # cached by signature, so a sim of another instance of the same graph
    # family and size takes it from the file without trials
    n = 30_000
    model = W.WORKLOADS["ba5_n1e6"]["model"]
    seeds = W.seed_nodes(n, 50, 6)
    cache = str(tmp_path / "tune.txt")
    runs = []
    for gseed in (4, 4):
        rp, ci = W.barabasi_albert(n, 5, gseed)
        with fs.Graph(rp, ci) as g:
            sim = fs.Sim.from_model(g, model, steps_per_graph=10, replicas=replicas)
            sim.seed(seeds, replica=-1)
            sim.step(30)
            before = [sim.get_state(r) for r in range(replicas)]
            res = sim.autotune(5, variants=True, cache_path=cache)
            assert sim.variant() == res["variant"]
            assert sim.bins()[:2] == (res["heavy_degree"], res["segment_edges"])
            for r in range(replicas):
                for x, y in zip(before[r], sim.get_state(r)):
                    np.testing.assert_array_equal(x, y)
            sim.step(40)
            runs.append((res, [(*sim.get_state(r)[:2], sim.history(0, 70, r)) for r in range(replicas)]))
            sim.close()
            ref = fs.Sim.from_model(g, model, heavy_degree=-1, replicas=replicas, variant=fs.VARIANT_STREAM)
            ref.seed(seeds, replica=-1)
            ref.step(70)
            plain = [(*ref.get_state(r)[:2], ref.history(0, 70, r)) for r in range(replicas)]
            ref.close()
        for a, b in zip(runs[-1][1], plain):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
    first, second = runs[0][0], runs[1][0]
    assert not first["from_cache"] and first["trials"] >= 3
    assert second["from_cache"] and second["signature"] == first["signature"]
    assert (second["variant"], second["heavy_degree"], second["segment_edges"]) == \
        (first["variant"], first["heavy_degree"], first["segment_edges"])
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith(first["signature"])


def test_autotune_adaptive_keeps_an_lds_variant():
    n = 20_000
    rp, ci = W.barabasi_albert(n, 4, 3)
    model = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.2, "dt": 0.1, "seed": 9}
    seeds = W.seed_nodes(n, 30, 2)
    out = []
    with fs.Graph(rp, ci) as g:
        for tune in (True, False):
            sim = fs.Sim.from_model(g, model, adaptive=True, epsilon=0.03, steps_per_graph=10)
            sim.seed(seeds, replica=0)
            sim.step(20)
            if tune:
                res = sim.autotune(4, variants=True)
                assert res["variant"] in ("resident", "summary")
            sim.step(30)
            out.append((sim.get_state(0)[:2], sim.history(0, 50), sim.step_sizes(0, 50)))
            sim.close()
    for x, y in zip(out[0], out[1]):
        if isinstance(x, tuple):
            for u, v in zip(x, y):
                np.testing.assert_array_equal(u, v)
        else:
            np.testing.assert_array_equal(x, y)


def test_compact_and_fp32_storage_agree_up_to_threshold_cases(small_graph):
    """The same state stepped once with FP32 ages in days and with compact
    step-count ages: the storages differ only in how the age is held (the
    float nearest n dt against n steps of dt), so their states may differ only
    at draws within the guard band of their FP64 threshold."""
    rp, ci, g = small_graph
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.2)
    rng = np.random.default_rng(8)
    st = rng.choice(4, n, p=[0.6, 0.15, 0.2, 0.05]).astype(np.int32)
    steps_age = rng.integers(0, 150, n).astype(np.uint16)
    days = (steps_age.astype(np.float64) * model["dt"]).astype(np.float32)
    got = {}
    for compact, age in [(False, days), (True, steps_age)]:
        sim = fs.Sim.from_model(g, model, storage=storage_of(compact))
        sim.set_state(st, age, 0, step_index=17)
        sim.step(1)
        got[compact] = sim.get_state(0)[0]
        sim.close()
    ora = oracle.step((rp, ci), model, st, steps_age, (st == 2).astype(np.float64), 17, compact=True)
    diff = np.flatnonzero(got[False] != got[True])
    for i in diff:
        assert ora["u"][i] >= 0 and abs(ora["u"][i] - ora["q"][i]) < 1e-5, (i, ora["u"][i], ora["q"][i])
    assert len(diff) <= 3
    assert (got[True] != st).sum() > 100     # the step moved many nodes
