"""The Markovian engine on the GPU (Section "Markovian engine", Algorithm
"Markovian Engine: One Tau-Leaping Step") against the FP64 oracle.

One step from a given state is compared node by node: states (a draw may
flip only within the guard band of its threshold, since tau and the
probability are FP32 on the device), the step size (FP32 against FP64), the
event count, and the influence, which must equal an exact recount from the
GPU's own new states whichever update mode ran.  Sparse pushes and full
recounts must give bit-identical trajectories, and so must captured replays
and eager launches.
"""
import numpy as np
import pytest

import oracle
import paper_2604_22092_amd as fs
import workloads as W
from _parity import check_mismatch_budget

pytestmark = pytest.mark.gpu

GUARD = 1e-6
MODELS = {
    "seir": {"model": "seir", "beta": 0.3, "sigma": 0.4, "gamma": 0.2},
    "sir": {"model": "sir", "beta": 0.25, "gamma": 0.15},
    "sis": {"model": "sis", "beta": 0.25, "gamma": 0.3},
}
STEP = {"theta": 0.01, "p_max": 0.1, "tau_max": 1.0}
GRAPHS = {}


def graph(name):
    if name not in GRAPHS:
        if name == "er":
            GRAPHS[name] = W.erdos_renyi(20_000, 8.0, 5)
        elif name == "ba":
            GRAPHS[name] = W.barabasi_albert(20_000, 4, 6)
        else:
            GRAPHS[name] = W.random_regular(10_000, 6, 7)
    return GRAPHS[name]


def events_between(a, b):
    return int(((a == 2) != (b == 2)).sum())


@pytest.mark.parametrize("mode", ["push", "recount"])
@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("gname", ["er", "ba"])
def test_one_step_matches_the_oracle(gname, model, mode):
    rp, ci = graph(gname)
    n = len(rp) - 1
    m = dict(MODELS[model], **STEP, seed=77)
    rng = np.random.default_rng(3)
    comps = [0, 1, 2, 3] if model == "seir" else [0, 2, 3] if model == "sir" else [0, 2]
    mism, total = 0, 0
    with fs.Graph(rp, ci) as g, fs.Markov(g, m, inertial_max=10**9 if mode == "push" else -1) as eng:
        for k, frac_i in [(0, 0.01), (9, 0.2), (123, 0.5)]:
            p = np.full(len(comps), (1 - frac_i) / (len(comps) - 1))
            p[comps.index(2)] = frac_i
            st = rng.choice(comps, n, p=p).astype(np.int32)
            eng.set_state(st, step_index=k, elapsed=1.5)
            eng.step(1)
            gst, ginf, kk, el = eng.get_state()
            assert kk == k + 1
            ora = oracle.markov_step((rp, ci), m, st, k)
            bad = [i for i in np.flatnonzero(gst != ora["state"])
                   if not (ora["u"][i] >= 0 and abs(ora["u"][i] - ora["p"][i]) < GUARD)]
            assert not bad, (k, bad[:5])
            mism += int((gst != ora["state"]).sum())
            total += n
            # the influence is exactly that of the GPU's new states (under SEIR
            # and SIR on the nodes that can still use it: the susceptible)
            want = oracle.markov_influence((rp, ci), gst)
            keep = np.ones(n, bool) if model == "sis" else gst == 0
            np.testing.assert_array_equal(ginf[keep], want[keep])
            counts, taus, evs = eng.history(k, 1)
            np.testing.assert_array_equal(counts[0], np.bincount(gst, minlength=4))
            assert taus[0] == pytest.approx(ora["tau"], rel=1e-6)
            assert el == pytest.approx(1.5 + ora["tau"], rel=1e-6)
            assert evs[0] == events_between(st, gst)
            assert ora["events"] > 0
    check_mismatch_budget(mism, total, f"{gname} {model} {mode}")


@pytest.mark.parametrize("model", list(MODELS))
def test_trajectory_matches_the_oracle(model):
    rp, ci = graph("er")
    n = len(rp) - 1
    m = dict(MODELS[model], **STEP, seed=11)
    seeds = W.seed_nodes(n, 20, 1)
    st0 = np.zeros(n, np.int32)
    st0[seeds] = 2
    steps = 400
    with fs.Graph(rp, ci) as g, fs.Markov(g, m, steps_per_graph=50, history_len=steps) as eng:
        eng.seed(seeds, fs.FS_I)
        eng.step(steps)
        gst, ginf, _, el = eng.get_state()
        gh, gt, ge = eng.history(0, steps)
    ost, oh, ot, oe = oracle.markov_run((rp, ci), m, st0, steps)
    # a divergence would have to start at a guard-band draw; none is expected
    np.testing.assert_array_equal(gh, oh)
    np.testing.assert_array_equal(gst, ost)
    np.testing.assert_allclose(gt, ot, rtol=1e-6)
    assert el == pytest.approx(ot.sum(), rel=1e-5)
    assert oh[:, 2].max() > 0.05 * n


@pytest.mark.parametrize("gname", ["er", "ba", "regular"])
def test_push_and_recount_and_replay_are_identical(gname):
    rp, ci = graph(gname)
    n = len(rp) - 1
    m = dict(MODELS["seir"], **STEP, seed=5)
    seeds = W.seed_nodes(n, 10, 2)
    out = []
    with fs.Graph(rp, ci) as g:
        for kw in [dict(inertial_max=10**9), dict(inertial_max=-1), dict(inertial_max=0, steps_per_graph=30),
                   dict(inertial_max=50, steps_per_graph=7)]:
            with fs.Markov(g, m, history_len=300, **kw) as eng:
                eng.seed(seeds, fs.FS_I)
                eng.step(137)
                eng.step(163)
                st, inf, k, el = eng.get_state()
                out.append((st, inf, *eng.history(0, 300), el))
    for o in out[1:]:
        np.testing.assert_array_equal(out[0][0], o[0])
        sus = out[0][0] == 0
        np.testing.assert_array_equal(out[0][1][sus], o[1][sus])   # influence of the susceptible
        for x, y in zip(out[0][2:], o[2:]):
            np.testing.assert_array_equal(x, y)
    assert out[0][2][:, 3].max() > 0.1 * n     # the epidemic ran


def test_no_infection_and_extinction():
    rp, ci = graph("regular")
    n = len(rp) - 1
    m = {**MODELS["sir"], **STEP, "tau_max": 0.5, "seed": 1}
    with fs.Graph(rp, ci) as g, fs.Markov(g, m, history_len=100) as eng:
        eng.step(20)       # nobody infectious: nothing happens, every step is the cap
        c, t, e = eng.history(0, 20)
        np.testing.assert_array_equal(c[:, 0], n)
        np.testing.assert_array_equal(t, np.float32(0.5))
        np.testing.assert_array_equal(e, 0)
        st = np.full(n, 3, np.int32)
        st[:5] = 2
        eng.set_state(st, step_index=20)
        eng.step(80)
        c, t, e = eng.history(20, 80)
        assert c[-1, 2] == 0 and c[-1, 3] == n   # the five recovered
        with pytest.raises(fs.FsError):
            eng.history(0, 30)                      # before the state load


def test_markov_rejections():
    rp, ci = graph("regular")
    w = np.ones(len(ci), np.float32)
    with fs.Graph(rp, ci, w) as g:
        with pytest.raises(fs.FsError):
            fs.Markov(g, dict(MODELS["sir"], **STEP))
    with fs.Graph(rp, ci) as g:
        for bad in [{**MODELS["sir"], **STEP, "theta": 0.0}, {**MODELS["sir"], **STEP, "gamma": -1.0}]:
            with pytest.raises(fs.FsError):
                fs.Markov(g, bad)
