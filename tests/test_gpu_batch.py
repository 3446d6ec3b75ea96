"""Batches of simulations and the scenario server: every member's and every
request's results equal the FP64 oracle's (whole trajectories per replica,
and one step from a fixed mid-epidemic state under the guard-band rule), and
equal those of the same simulation run alone.

The members differ in graph family and size (random regular, Erdos-Renyi,
Barabasi-Albert with degree-binned hub rows), holding-time laws, beta, dt,
seed and replica count, like the requests of a serving mix.
"""
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W
from _parity import check_mismatch_budget, check_one_step

pytestmark = pytest.mark.gpu

SCEN = [
    # (graph spec, laws/rates, replicas, seeds)
    (("regular", 6000, 8, 1), {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.09, "dt": 0.1, "seed": 3}, 4, 8),
    (("ba", 20000, 4, 2), {"ei": ("erlang", 3, 1.0), "ir": ("weibull", 2.0, 6.0), "beta": 0.05,
                           "dt": 0.1, "seed": 7}, 1, 20),
    (("er", 5000, 10.0, 3), {"ei": ("exp", 0.3), "ir": ("lognormal", 1.2, 0.5), "beta": 0.08,
                             "dt": 0.2, "seed": 11}, 16, 5),
    (("regular", 3000, 4, 4), {"ei": ("weibull", 1.5, 3.0), "ir": ("erlang", 2, 0.4),
                               "beta": 0.2, "dt": 0.05, "seed": 2**40 + 1}, 2, 6),
]


@pytest.fixture(scope="module")
def graphs():
    out = []
    for spec, _, _, _ in SCEN:
        rp, ci = W.workload_graph(spec)
        out.append((rp, ci, fs.Graph(rp, ci)))
    yield out
    for _, _, g in out:
        g.close()


def new_sim(g, model, R, storage=fs.FS_STORAGE_FP32, variant=fs.VARIANT_STREAM, **kw):
    return fs.Sim.from_model(g, model, replicas=R, storage=storage, variant=variant, **kw)


def snapshot(sim, steps):
    return [(*sim.get_state(r)[:2], sim.history(0, steps, r)) for r in range(sim.replicas)]


def alone(g, rp, model, R, nseed, steps, storage, variant=fs.VARIANT_AUTO):
    sim = new_sim(g, model, R, storage, variant=variant)
    sim.seed(W.seed_nodes(len(rp) - 1, nseed, 5), replica=-1)
    sim.step(steps)
    out = snapshot(sim, steps)
    sim.close()
    return out


def assert_same(a, b, label):
    for r, (x, y) in enumerate(zip(a, b)):
        for u, v, what in zip(x, y, ["state", "age", "history"]):
            np.testing.assert_array_equal(u, v, err_msg=f"{label} replica {r} {what}")


def oracle_trajectory(rp, ci, model, nseed, steps, replica, compact, weights=None):
    """The oracle's (state, age, history) of one replica from the seeded start."""
    n = len(rp) - 1
    graph = (rp, ci) if weights is None else (rp, ci, weights)
    age = np.zeros(n, np.uint16 if compact else np.float32)
    return oracle.run(graph, model, W.initial_state(n, W.seed_nodes(n, nseed, 5)), age, steps,
                      replica=replica, compact=compact)


def assert_matches_oracle(got, rp, ci, model, nseed, steps, compact, label, weights=None):
    """got: per replica (state, age, history) of a GPU run from the seeded
    start.  A divergence would have to start at a guard-band draw (about 1e-3
    expected over all these runs), so whole trajectories compare exactly."""
    for r, (gst, gage, ghist) in enumerate(got):
        ost, oage, ohist = oracle_trajectory(rp, ci, model, nseed, steps, r, compact, weights)
        np.testing.assert_array_equal(ghist, ohist, err_msg=f"{label} replica {r} history")
        np.testing.assert_array_equal(gst, ost, err_msg=f"{label} replica {r} state")
        np.testing.assert_array_equal(gage, oage, err_msg=f"{label} replica {r} age")


def test_packed_sim_joins_a_batch_with_plain_columns(graphs):
    # a single-replica sim of a uniform unweighted graph starts with packed
    # columns; joining a batch moves it to 32-bit columns (the batch step
    # reads those) with its trajectory unchanged: equal to the packed solo
    # run and to the oracle
    (rp, ci, g), (_, m, _, ns) = graphs[0], SCEN[0]
    steps = 60
    ref = alone(g, rp, m, 1, ns, steps, fs.FS_STORAGE_FP32, variant=fs.VARIANT_STREAM)
    with fs.Batch(fs.FS_STORAGE_FP32) as b:
        s = new_sim(g, m, 1)
        assert s.column_bits() == 20
        s.seed(W.seed_nodes(len(rp) - 1, ns, 5), replica=-1)
        s.step(10)  # some steps alone with packed columns first
        b.add(s)
        assert s.column_bits() == 32
        b.step(steps - 10)
        b.sync()
        got = snapshot(s, steps)
        b.remove(s)
        s.close()
    assert_same(got, ref, "packed member")
    assert_matches_oracle(got, rp, ci, m, ns, steps, False, "packed member")


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
def test_batch_members_equal_alone(graphs, compact):
    storage = fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32
    steps = 120
    ref = [alone(g, rp, m, R, ns, steps, storage) for (rp, _, g), (_, m, R, ns) in zip(graphs, SCEN)]
    with fs.Batch(storage) as b:
        sims = []
        for (rp, _, g), (_, m, R, ns) in zip(graphs, SCEN):
            s = new_sim(g, m, R, storage)
            s.seed(W.seed_nodes(len(rp) - 1, ns, 5), replica=-1)
            b.add(s)
            sims.append(s)
        assert b.size() == len(SCEN)
        for _ in range(3):
            b.step(steps // 3)
        b.sync()
        got = [snapshot(s, steps) for s in sims]
        for s in sims:
            b.remove(s)
            s.close()
    for i, (x, y) in enumerate(zip(got, ref)):
        assert_same(x, y, f"member {i}")
    # every member, every replica: the oracle's trajectory
    for i, (x, (rp, ci, _), (_, m, R, ns)) in enumerate(zip(got, graphs, SCEN)):
        assert_matches_oracle(x, rp, ci, m, ns, steps, compact, f"member {i}")
    # the epidemics moved
    assert all(h[-1, 0] < len(rp) - 1 for ((_, _, h), *_), (rp, _, _) in zip(got, graphs))


def mid_epidemic_state(n, rng, dt, compact):
    """A state with every compartment present and ages of both kinds: the
    ages steps reach (m steps of dt, summed in FP32) and arbitrary ones."""
    st = rng.choice(4, size=n, p=[0.55, 0.15, 0.2, 0.1]).astype(np.int32)
    m = rng.integers(0, 150, n)
    if compact:
        return st, m.astype(np.uint16)
    table = np.zeros(151, np.float32)
    for j in range(1, 151):
        table[j] = np.float32(table[j - 1] + np.float32(dt))
    age = table[m]
    odd = rng.random(n) < 0.3
    age[odd] = (rng.random(odd.sum()) * 20.0).astype(np.float32)
    return st, age


@pytest.mark.parametrize("compact", [False, True], ids=["fp32", "compact"])
def test_batch_one_step_matches_oracle(graphs, compact):
    # every member from its own mid-epidemic state in every replica, one step
    # of the batch launch (member lookup by block range), against the oracle
    # node by node: states up to guard-band draws, ages, FP32 rates within
    # the hazard tolerance
    storage = fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32
    rng = np.random.default_rng(7)
    total, flips = 0, 0
    with fs.Batch(storage) as b:
        sims, states = [], []
        for (rp, _, g), (_, m, R, _) in zip(graphs, SCEN):
            s = new_sim(g, m, R, storage, record_rates=True)
            per = [mid_epidemic_state(len(rp) - 1, rng, m["dt"], compact) for _ in range(R)]
            for r, (st, age) in enumerate(per):
                s.set_state(st, age, r, step_index=37 if r == 0 else -1)
            b.add(s)
            sims.append(s)
            states.append(per)
        b.step(1)
        b.sync()
        for i, (s, per, (rp, ci, _), (_, m, R, _)) in enumerate(zip(sims, states, graphs, SCEN)):
            for r, (st, age) in enumerate(per):
                gst, gage, gk = s.get_state(r)
                assert gk == 38
                iota = (st == 2).astype(np.float64)
                ora = oracle.step((rp, ci), m, st, age, iota, 37, replica=r, compact=compact)
                nm, _ = check_one_step({"state": gst, "age": gage, "rates": s.rates(r)}, ora, st,
                                       f"member {i} replica {r}")
                flips += nm
                total += len(st)
        for s in sims:
            b.remove(s)
            s.close()
    check_mismatch_budget(flips, total, "batch one step")


def test_batch_membership_changes_mid_run(graphs):
    (rp0, _, g0), (rp1, _, g1) = graphs[0], graphs[1]
    (_, m0, R0, n0), (_, m1, R1, n1) = SCEN[0], SCEN[1]
    ref0 = alone(g0, rp0, m0, R0, n0, 90, fs.FS_STORAGE_FP32)
    ref1 = alone(g1, rp1, m1, R1, n1, 50, fs.FS_STORAGE_FP32)
    with fs.Batch() as b:
        a = new_sim(g0, m0, R0)
        a.seed(W.seed_nodes(len(rp0) - 1, n0, 5), replica=-1)
        b.add(a)
        b.step(40)
        c = new_sim(g1, m1, R1)
        c.seed(W.seed_nodes(len(rp1) - 1, n1, 5), replica=-1)
        b.add(c)                      # joins at its own step 0
        b.step(50)
        b.remove(c)
        got1 = snapshot(c, 50)
        c.close()
        assert a.step_index() == 90
        got0 = snapshot(a, 90)
        b.remove(a)
        a.step(5)                     # back on its own stream, steps alone again
        assert a.step_index() == 95
        a.close()
    assert_same(got0, ref0, "early member")
    assert_same(got1, ref1, "late member")


def test_batch_member_rules(graphs):
    rp, _, g = graphs[0]
    _, m, R, _ = SCEN[0]
    with fs.Batch() as b:
        res = new_sim(g, m, R, variant=fs.VARIANT_RESIDENT)
        with pytest.raises(fs.FsError):
            b.add(res)                                   # not the streaming variant
        res.close()
        cmp_ = new_sim(g, m, R, storage=fs.FS_STORAGE_COMPACT)
        with pytest.raises(fs.FsError):
            b.add(cmp_)                                  # storage differs
        cmp_.close()
        s = new_sim(g, m, R)
        b.add(s)
        with pytest.raises(fs.FsError) as ei:
            s.step(1)                                    # stepped by the batch only
        assert ei.value.status == 5
        with pytest.raises(fs.FsError):
            s.close()
        with pytest.raises(fs.FsError):
            b.add(s)                                     # already a member
        b.remove(s)
        s.close()
        b.step(3)                                        # empty batch: no work


# ------------------------------------------------------------------ server

def request_set(graphs, k, rng):
    out = []
    for i in range(k):
        j = i % len(SCEN)
        _, m, R, ns = SCEN[j]
        m = dict(m, seed=int(rng.integers(0, 2**63)), beta=m["beta"] * float(rng.uniform(0.8, 1.25)))
        steps = int(rng.integers(40, 160))
        out.append((j, m, R, ns, steps))
    return out


def test_server_results_equal_alone(graphs):
    rng = np.random.default_rng(42)
    reqs = request_set(graphs, 12, rng)
    with fs.Server(max_active=6, steps_per_round=16) as sv:
        ids = [None] * len(reqs)

        def submitter():
            # staggered arrivals: later requests land while earlier ones run
            for i, (j, m, R, ns, steps) in enumerate(reqs):
                rp, _, g = graphs[j]
                ids[i] = sv.submit(g, m["ei"], m["ir"], m["beta"], m["dt"], m["seed"], R, steps,
                                   W.seed_nodes(len(rp) - 1, ns, 5))
                time.sleep(0.002 * (i % 3))

        t = threading.Thread(target=submitter)
        t.start()
        t.join()
        results = []
        for i in ids:
            assert sv.wait(i, 120.0)
            results.append(sv.result(i))
        st = sv.stats()
        assert st["queued"] == 0 and st["active"] == 0 and st["rounds"] > 0
    overlapped = 0
    for (j, m, R, ns, steps), (hist, info) in zip(reqs, results):
        rp, ci, g = graphs[j]
        ref = alone(g, rp, m, R, ns, steps, fs.FS_STORAGE_FP32)
        for r in range(R):
            np.testing.assert_array_equal(hist[:, r, :], ref[r][2], err_msg=f"request scenario {j} replica {r}")
            # and the oracle's per-step counts of the same replica
            _, _, ohist = oracle_trajectory(rp, ci, m, ns, steps, r, False)
            np.testing.assert_array_equal(hist[:, r, :], ohist, err_msg=f"request scenario {j} replica {r} (oracle)")
        assert info["status"] == 0 and info["t_submit"] <= info["t_admit"] <= info["t_done"]
        assert info["n_steps"] == steps and info["n_replicas"] == R
    # requests overlapped on the device: some admission happened before an
    # earlier request had finished
    spans = sorted((info["t_admit"], info["t_done"]) for _, info in results)
    overlapped = sum(1 for a, b in zip(spans, spans[1:]) if b[0] < a[1])
    assert overlapped > 0


def test_server_budget_slots_and_errors(graphs):
    rp, _, g = graphs[2]
    _, m, R, ns = SCEN[2]
    seeds = W.seed_nodes(len(rp) - 1, ns, 5)
    with fs.Server(memory_budget=64 << 20, max_active=1, steps_per_round=7) as sv:
        big = fs.Graph(*W.random_regular_matchings(2_000_000, 8, 9))
        with pytest.raises(fs.FsError) as ei:
            sv.submit(big, m["ei"], m["ir"], m["beta"], m["dt"], 1, 16, 100, [0])
        assert ei.value.status == 6                   # FS_ERR_BUDGET
        bad = sv.submit(g, ("weibull", 0.5, 2.0), m["ir"], m["beta"], m["dt"], 1, R, 10, seeds)
        good = [sv.submit(g, m["ei"], m["ir"], m["beta"], m["dt"], s, R, 30, seeds) for s in range(3)]
        assert sv.wait(bad, 60.0)
        with pytest.raises(fs.FsError) as ei:
            sv.result(bad)
        assert ei.value.status == 1                   # the law is rejected at admission
        infos = []
        for s, rid in enumerate(good):
            assert sv.wait(rid, 60.0)
            hist, info = sv.result(rid)
            infos.append(info)
            ref = alone(g, rp, dict(m, seed=s), R, ns, 30, fs.FS_STORAGE_FP32)
            for r in range(R):
                np.testing.assert_array_equal(hist[:, r, :], ref[r][2])
        # one slot: the requests ran one after another, in submission order
        # (the next one's sim may be created while the previous one's last
        # round runs, but it steps only after that)
        for a, b in zip(infos, infos[1:]):
            assert b["t_admit"] > a["t_admit"] and b["t_done"] > a["t_done"]
        with pytest.raises(fs.FsError):
            sv.result(good[0])                        # already collected
    big.close()


def test_server_mixes_weighted_and_unit_weight_requests(graphs):
    # small requests on a weighted graph and on unit-weight graphs arrive
    # together: each runs in the batch of its own kind and gets its solo
    # results and the oracle's
    rp, ci = W.random_regular(4000, 6, 12)
    w = (0.5 + np.random.default_rng(3).random(len(ci))).astype(np.float32)
    model = {"ei": W.LN_E, "ir": ("weibull", 2.0, 5.0), "beta": 0.12, "dt": 0.1, "seed": 99}
    steps, R, ns = 60, 2, 12
    with fs.Graph(rp, ci, w) as gw:
        ref_w = alone(gw, rp, model, R, ns, steps, fs.FS_STORAGE_FP32, variant=fs.VARIANT_STREAM)
        with fs.Server(max_active=8, steps_per_round=9) as sv:
            ids = []
            for i in range(6):
                if i % 2 == 0:
                    ids.append(("w", sv.submit(gw, model["ei"], model["ir"], model["beta"], model["dt"],
                                               model["seed"], R, steps, W.seed_nodes(len(rp) - 1, ns, 5))))
                else:
                    rq, _, gq = graphs[0]
                    _, mq, Rq, nsq = SCEN[0]
                    ids.append(("u", sv.submit(gq, mq["ei"], mq["ir"], mq["beta"], mq["dt"], mq["seed"], Rq,
                                               steps, W.seed_nodes(len(rq) - 1, nsq, 5))))
            out = []
            for kind, rid in ids:
                assert sv.wait(rid, 120.0)
                out.append((kind, sv.result(rid)[0]))
    rq, cq, gq = graphs[0]
    _, mq, Rq, nsq = SCEN[0]
    ref_u = alone(gq, rq, mq, Rq, nsq, steps, fs.FS_STORAGE_FP32)
    for kind, hist in out:
        ref = ref_w if kind == "w" else ref_u
        for r in range(hist.shape[1]):
            np.testing.assert_array_equal(hist[:, r, :], ref[r][2], err_msg=f"{kind} replica {r}")
    for r in range(R):
        _, _, ohist = oracle_trajectory(rp, ci, model, ns, steps, r, False, weights=w)
        np.testing.assert_array_equal(ref_w[r][2], ohist, err_msg=f"weighted replica {r} (oracle)")
    assert ref_w[0][2][-1, 0] < len(rp) - 1  # the weighted epidemic moved
