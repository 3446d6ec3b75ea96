"""The device memory hook (fs_set_allocator): with PyTorch's caching
allocator behind it, graphs, sims and Markovian engines take their arrays
from PyTorch (visible in torch.cuda.memory_allocated), return every block
when they are released, and compute exactly what they compute on the
library's own allocator."""
import numpy as np
import pytest
import torch  # (at collection, before any test loads the library: one HIP runtime for both)

import paper_2604_22092_amd as fs
import workloads as W

pytestmark = pytest.mark.gpu

MODEL = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.12, "dt": 0.1, "seed": 3}
MARKOV = {"model": "sir", "beta": 0.25, "gamma": 0.15, "theta": 0.01, "p_max": 0.1, "tau_max": 1.0, "seed": 4}


def run(rp, ci, seeds, probe=None):
    with fs.Graph(rp, ci) as g:
        sim = fs.Sim.from_model(g, MODEL, steps_per_graph=20, replicas=2)
        sim.seed(seeds)
        sim.step(120)
        eng = fs.Markov(g, MARKOV, steps_per_graph=20, history_len=120)
        eng.seed(seeds, fs.FS_I)
        eng.step(120)
        if probe:
            probe()
        out = (sim.get_state(0)[:2], sim.history(0, 120, 1), eng.get_state()[0], eng.history(0, 120)[0])
        eng.close()
        sim.close()
    return out


def test_torch_caching_allocator_backs_the_library():
    assert len(fs.hip_runtimes()) <= 1
    rp, ci = W.barabasi_albert(30_000, 4, 2)   # degree-sorted order and heavy rows too
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 20, 1)
    ref = run(rp, ci, seeds)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    seen = []
    fs.use_torch_allocator(0)
    try:
        got = run(rp, ci, seeds, probe=lambda: seen.append(torch.cuda.memory_allocated(0)))
    finally:
        fs.set_allocator()
    torch.cuda.synchronize()
    assert seen[0] > before + 8 * n * 2          # at least the sim's state and age
    assert torch.cuda.memory_allocated(0) == before   # every block returned
    for a, b in zip(ref, got):
        if isinstance(a, tuple):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
        else:
            np.testing.assert_array_equal(a, b)
    # and the library's own allocator serves again
    again = run(rp, ci, seeds)
    np.testing.assert_array_equal(again[1], ref[1])
