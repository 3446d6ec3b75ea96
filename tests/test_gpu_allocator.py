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


class CountingHook:
    """A device allocator that serves `grant` blocks from PyTorch's caching
    allocator and then returns NULL, and tracks the blocks it has out."""

    def __init__(self, grant):
        self.grant = grant
        self.live = {}
        self.calls = 0

    def alloc(self, nbytes):
        self.calls += 1
        if self.grant == 0:
            return 0
        self.grant -= 1
        p = torch.cuda.caching_allocator_alloc(nbytes, device=0)
        self.live[p] = nbytes
        return p

    def free(self, p):
        assert p in self.live, "freed a block this allocator did not give out"
        del self.live[p]
        torch.cuda.caching_allocator_delete(p)


def test_failing_allocator_gives_out_of_memory_and_leaks_nothing():
    # every allocation of fs_graph_create and of fs_sim_create fails in turn:
    # FS_ERR_OUT_OF_MEMORY, *out stays NULL, and every block the allocator
    # gave out before the failure has come back
    import ctypes

    L = fs.lib()
    rp, ci = W.barabasi_albert(5000, 3, 4)
    w = np.ones(len(ci), np.float32)
    rp32, ci32 = rp.astype(np.int32), ci.astype(np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for grant in range(0, 10):
        hook = CountingHook(grant)
        fs.set_allocator(hook.alloc, hook.free)
        try:
            h = ctypes.c_void_p()
            st = L.fs_graph_create(len(rp) - 1, ptr(rp32), ptr(ci32), ptr(w), ctypes.byref(h))
        finally:
            fs.set_allocator()
        if st == 0:
            assert grant >= 4  # row_ptr, col_ind, node ids, weights
            fs.fs_graph_destroy(h)
            assert not hook.live
            break
        assert st == 3 and h.value is None, (grant, st)
        assert hook.calls == grant + 1 and not hook.live, grant
    else:
        raise AssertionError("fs_graph_create never succeeded")

    succeeded = False
    for grant in range(0, 64):
        with fs.Graph(rp, ci) as g:
            hook = CountingHook(grant)
            p = fs.make_params(W.LN_E, W.LN_I, 0.1, 0.1, replicas=4, steps_per_graph=10, record_rates=True,
                               heavy_degree=16, segment_edges=64)
            fs.set_allocator(hook.alloc, hook.free)
            try:
                h = ctypes.c_void_p()
                st = L.fs_sim_create(g.handle, ctypes.byref(p), ctypes.byref(h))
            finally:
                fs.set_allocator()
            if st == 0:
                fs.fs_sim_destroy(h)
                succeeded = True
            else:
                assert st == 3 and h.value is None, (grant, st)
                assert hook.calls == grant + 1, grant
        # the sim's blocks, and the graph's layout built through the hook,
        # are all back once the graph is released
        torch.cuda.synchronize()
        assert not hook.live, (grant, len(hook.live))
        if succeeded:
            assert grant >= 5
            break
    assert succeeded
