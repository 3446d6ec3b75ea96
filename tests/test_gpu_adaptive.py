"""Adaptive step size on the GPU (Section "Bernoulli tau-leaping", adaptive
step selection; the tau update of Algorithm 3) against the FP64 oracle.

The GPU takes each step's size from its own FP32 rates, so trajectories are
compared step by step with the oracle fed the GPU's step sizes, the size rule
is checked against the oracle's FP64 rates, and whole adaptive trajectories
are compared by their statistics.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W
from _parity import check_mismatch_budget, check_one_step

pytestmark = pytest.mark.gpu

SMALL = W.WORKLOADS["regular10_n1e4"]
EPS, CAP = 0.03, 0.1


@pytest.fixture(scope="module")
def small():
    rp, ci = W.workload_graph(SMALL["graph"])
    with fs.Graph(rp, ci) as g:
        yield rp, ci, g


def new_sim(g, model, **kw):
    kw.setdefault("adaptive", True)
    kw.setdefault("epsilon", EPS)
    return fs.Sim.from_model(g, dict(model, dt=CAP), **kw)


@pytest.mark.parametrize("variant", [fs.VARIANT_RESIDENT, fs.VARIANT_SUMMARY], ids=["resident", "summary"])
def test_one_step_parity_with_the_gpu_step_sizes(small, variant):
    rp, ci, g = small
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.1)
    seeds = W.seed_nodes(n, 20, 4)
    sim = new_sim(g, model, record_rates=True, variant=variant)
    total, mism = 0, 0
    try:
        sim.seed(seeds)
        for k0 in [0, 60, 150, 300]:
            sim.step(k0 - sim.step_index())
            st, age, k = sim.get_state(0)
            sim.step(1)
            gst, gage, _ = sim.get_state(0)
            dt_k = sim.step_sizes(k, 1)[0]
            if k0 == 0:
                assert dt_k == np.float32(CAP)     # the first step is the cap
            ora = oracle.step((rp, ci), dict(model, dt=dt_k), st, age, (st == 2).astype(np.float64), k)
            nm, _ = check_one_step({"state": gst, "age": gage, "rates": sim.rates(0)}, ora, st, f"k={k}")
            total += n
            mism += nm
            # the next step's size follows the rule from this step's largest rate
            sim.step(1)
            dt_next = sim.step_sizes(k + 1, 1)[0]
            want = oracle.next_dt(ora["lam"].max(), EPS, CAP)
            assert dt_next == pytest.approx(want, rel=1e-5), (k, dt_next, want)
            if k0 > 0:
                assert ora["lam"].max() > 0   # (at step 0 every seed is at age 0: all rates 0)
    finally:
        sim.close()
    check_mismatch_budget(mism, total, "adaptive checkpoints")


def test_huge_epsilon_reproduces_the_fixed_step_run(small):
    rp, ci, g = small
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 10, 5)
    out = []
    for adaptive in [False, True]:
        sim = fs.Sim.from_model(g, dict(SMALL["model"], dt=CAP), adaptive=adaptive, epsilon=1e9,
                                steps_per_graph=40)
        sim.seed(seeds)
        sim.step(200)
        out.append((*sim.get_state(0)[:2], sim.history(0, 200), sim.step_sizes(0, 200)))
        sim.close()
    for x, y in zip(out[0], out[1]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(out[1][3], np.float64(np.float32(CAP)))


def test_graph_replay_equals_eager_and_restart_after_state_load(small):
    rp, ci, g = small
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.12)
    seeds = W.seed_nodes(n, 15, 6)
    res = []
    for b in [0, 25]:
        sim = new_sim(g, model, steps_per_graph=b)
        sim.seed(seeds)
        sim.step(137)
        res.append((*sim.get_state(0)[:2], sim.history(0, 137), sim.step_sizes(0, 137)))
        sim.close()
    for x, y in zip(res[0], res[1]):
        np.testing.assert_array_equal(x, y)
    dts = res[0][3]
    assert dts.min() < CAP * 0.99 and dts.max() <= np.float32(CAP)   # the rule engaged
    # a state load restarts the rule: the next step is the cap again
    sim = new_sim(g, model)
    sim.set_state(res[0][0], res[0][1], 0, step_index=137)
    sim.step(2)
    d = sim.step_sizes(137, 2)
    assert d[0] == np.float32(CAP) and d[1] < CAP
    sim.close()


def test_adaptive_ensemble_matches_the_oracle(small):
    """Peak prevalence, attack rate and elapsed time of adaptive runs: 24 GPU
    sims against 24 oracle runs (other Philox seeds), 3 standard errors."""
    rp, ci, g = small
    n = len(rp) - 1
    model = dict(SMALL["model"], beta=0.09)
    seeds = W.seed_nodes(n, 20, 7)
    steps, R = 600, 24

    def stats(hist, dts):
        return hist[:, 2].max() / n, 1 - hist[-1, 0] / n, dts.sum()

    gpu, ora = [], []
    for r in range(R):
        sim = new_sim(g, dict(model, seed=1000 + r), history_len=steps)
        sim.seed(seeds)
        sim.step(steps)
        gpu.append(stats(sim.history(0, steps), sim.step_sizes(0, steps)))
        sim.close()
        _, _, h, d = oracle.run_adaptive((rp, ci), dict(model, seed=5000 + r), W.initial_state(n, seeds),
                                         np.zeros(n, np.float32), steps, EPS, CAP)
        ora.append(stats(h, d))
    gpu, ora = np.array(gpu), np.array(ora)
    for j, name in enumerate(["peak", "attack rate", "elapsed days"]):
        a, b = gpu[:, j], ora[:, j]
        se = math.sqrt(a.var(ddof=1) / R + b.var(ddof=1) / R)
        assert abs(a.mean() - b.mean()) < 3 * se + 1e-12, (name, a.mean(), b.mean(), se)
    assert gpu[:, 1].mean() > 0.3


def test_adaptive_rejections(small):
    rp, ci, g = small
    m = SMALL["model"]
    for kw in [dict(storage=fs.FS_STORAGE_COMPACT), dict(variant=fs.VARIANT_STREAM), dict(epsilon=0.0)]:
        with pytest.raises(fs.FsError) as ei:
            new_sim(g, m, **kw)
        assert ei.value.status == 1
    sim = new_sim(g, m, variant=fs.VARIANT_RESIDENT)
    with fs.Batch() as b:
        with pytest.raises(fs.FsError):
            b.add(sim)   # not the streaming variant, and adaptive
    sim.close()
    with fs.Server() as sv:
        with pytest.raises(fs.FsError):
            fs.fs_server_submit(sv.handle, g.handle, fs.make_params(m["ei"], m["ir"], 0.1, 0.1, 1, 1,
                                                                    adaptive=True), 10, [0])
