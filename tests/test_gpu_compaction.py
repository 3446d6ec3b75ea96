"""Active-node compaction on the GPU (Section "Epidemic-aware compute
sparsity: active-node compaction"; Table "compaction_summary").

Compaction only skips work whose outcome is fixed (64-unit chunks whose
units are all R, an absorbing state), so against the same run without it
every per-step count, every final state, every age of a unit that is not R
and every recorded rate must be bit-identical; only the ages of R units in
skipped chunks stop advancing.  The runs below saturate (most nodes end in
R), so many chunks are skipped, which the frozen R ages confirm.
"""
import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = {"stream": fs.VARIANT_STREAM, "resident": fs.VARIANT_RESIDENT, "summary": fs.VARIANT_SUMMARY}
MODEL = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.4, "dt": 0.2, "seed": 19}


def ba_graph():
    rp, ci = W.barabasi_albert(30_000, 4, 8)
    return rp, ci, None


def regular_graph():
    rp, ci = W.random_regular(20_000, 8, 6)
    return rp, ci, None


def weighted_graph():
    rp, ci = W.random_regular(16_000, 6, 2)
    return rp, ci, np.random.default_rng(4).uniform(0.5, 1.5, len(ci)).astype(np.float32)


def run(g, n, seeds, steps, compaction, replicas=1, variant=0, b=0, compact=False, model=MODEL,
        rates=False, chunks=1):
    sim = fs.Sim.from_model(g, model, compaction=compaction, replicas=replicas, variant=variant,
                            steps_per_graph=b, record_rates=rates,
                            storage=fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32,
                            history_len=steps)
    sim.seed(seeds)
    per = steps // chunks
    for _ in range(chunks):
        sim.step(per)
    out = {"hist": [sim.history(0, per * chunks, r) for r in range(replicas)],
           "state": [sim.get_state(r) for r in range(replicas)],
           "rates": [sim.rates(r) for r in range(replicas)] if rates else None}
    sim.close()
    return out


def assert_same(ref, cmp, replicas, rates=False):
    frozen = 0
    for r in range(replicas):
        np.testing.assert_array_equal(ref["hist"][r], cmp["hist"][r])
        st0, age0, k0 = ref["state"][r]
        st1, age1, k1 = cmp["state"][r]
        assert k0 == k1
        np.testing.assert_array_equal(st0, st1)
        live = st0 != fs.FS_R
        np.testing.assert_array_equal(age0[live], age1[live])
        # R ages of skipped chunks stopped: never ahead of the full run's
        assert np.all(age1[~live] <= age0[~live])
        frozen += int((age1[~live] < age0[~live]).sum())
        if rates:
            np.testing.assert_array_equal(ref["rates"][r], cmp["rates"][r])
    return frozen


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("gname", ["ba", "regular"])
def test_compaction_is_exact(gname, variant):
    rp, ci, w = ba_graph() if gname == "ba" else regular_graph()
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 20, 1)
    steps = 400
    with fs.Graph(rp, ci, w) as g:
        ref = run(g, n, seeds, steps, False, variant=VARIANTS[variant], b=25, rates=True)
        cmp = run(g, n, seeds, steps, True, variant=VARIANTS[variant], b=25, rates=True)
    frozen = assert_same(ref, cmp, 1, rates=True)
    final = ref["hist"][0][-1]
    print(f"[compaction] {gname} {variant}: final {final.tolist()}, frozen R ages {frozen}")
    assert final[3] > 0.8 * n
    assert frozen > 0.2 * n      # most R units sat in skipped chunks


@pytest.mark.parametrize("replicas,variant,b,compact", [
    (4, "resident", 0, False), (4, "stream", 10, True), (16, "summary", 7, False), (2, "stream", 0, True)])
def test_compaction_replicas_and_launch_modes(replicas, variant, b, compact):
    rp, ci, w = ba_graph()
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 20, 3)
    with fs.Graph(rp, ci, w) as g:
        ref = run(g, n, seeds, 300, False, replicas, VARIANTS[variant], b, compact, chunks=3)
        cmp = run(g, n, seeds, 300, True, replicas, VARIANTS[variant], b, compact, chunks=3)
    frozen = assert_same(ref, cmp, replicas)
    assert frozen > 0


def test_compaction_weighted_and_shedding_match_the_oracle():
    rp, ci, w = weighted_graph()
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 15, 5)
    model = dict(MODEL, beta=0.6, shed=("density", ("lognormal", 1.0, 0.5), 4.0))
    steps = 300
    with fs.Graph(rp, ci, w) as g:
        ref = run(g, n, seeds, steps, False, b=20, model=model)
        cmp = run(g, n, seeds, steps, True, b=20, model=model)
    assert_same(ref, cmp, 1)
    # and the epidemic is the oracle's (the same draws: only a guard-band
    # flip of an FP32 threshold could make the two drift apart a little)
    _, _, oh = oracle.run((rp, ci, w), model, W.initial_state(n, seeds), np.zeros(n, np.float32), steps)
    assert np.abs(cmp["hist"][0] - oh).max() <= 0.01 * n
    assert oh[-1, 3] > 0.5 * n


def test_state_load_and_seeding_revive_skipped_chunks():
    rp, ci, w = ba_graph()
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 20, 7)
    rng = np.random.default_rng(0)
    with fs.Graph(rp, ci, w) as g:
        sims = [fs.Sim.from_model(g, MODEL, compaction=c, steps_per_graph=10, history_len=1000)
                for c in (False, True)]
        for s in sims:
            s.seed(seeds)
            s.step(300)
        st, age, k = sims[0].get_state(0)
        assert (st == fs.FS_R).mean() > 0.8
        # revive: a tenth of the recovered nodes back to S, a few of them exposed
        back = np.flatnonzero(st == fs.FS_R)
        back = rng.choice(back, len(back) // 10, replace=False)
        st2 = st.copy()
        st2[back] = fs.FS_S
        for s in sims:
            s.set_state(st2, age, 0)
            s.seed(back[:5])
            s.step(200)
        a, b = sims[0].get_state(0), sims[1].get_state(0)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(sims[0].history(300, 200), sims[1].history(300, 200))
        live = a[0] != fs.FS_R
        np.testing.assert_array_equal(a[1][live], b[1][live])
        # the revived epidemic spread again
        assert sims[0].history(300, 200)[:, 1:3].sum() > 0
        # seeding into chunks that were skipped (R nodes straight to E)
        r_nodes = np.flatnonzero(a[0] == fs.FS_R)[:50]
        for s in sims:
            s.seed(r_nodes)
            s.step(60)
        np.testing.assert_array_equal(sims[0].get_state(0)[0], sims[1].get_state(0)[0])
        np.testing.assert_array_equal(sims[0].history(500, 60), sims[1].history(500, 60))
        for s in sims:
            s.close()


def test_compaction_with_adaptive_steps_and_tuning():
    rp, ci, w = ba_graph()
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 20, 11)
    out = []
    with fs.Graph(rp, ci, w) as g:
        for c in (False, True):
            sim = fs.Sim.from_model(g, dict(MODEL, dt=0.25), compaction=c, adaptive=True, epsilon=0.05,
                                    steps_per_graph=16)
            sim.seed(seeds)
            sim.step(100)
            sim.tune(4)   # snapshots and restores everything, compaction state included
            sim.step(250)
            out.append((sim.get_state(0), sim.history(0, 350), sim.step_sizes(0, 350)))
            sim.close()
    (s0, h0, d0), (s1, h1, d1) = out
    np.testing.assert_array_equal(s0[0], s1[0])
    np.testing.assert_array_equal(h0, h1)
    np.testing.assert_array_equal(d0, d1)


def test_compaction_rejections():
    rp, ci, w = regular_graph()
    with fs.Graph(rp, ci, w) as g:
        sim = fs.Sim.from_model(g, MODEL, compaction=True, variant=fs.VARIANT_STREAM)
        with fs.Batch() as b:
            with pytest.raises(fs.FsError):
                b.add(sim)
        sim.close()
