"""fs_sim_seed_noalloc (seeding with the node list staged in the library's
fixed device array) against fs_sim_seed: the same states after each call,
and the same trajectories after it, on two calls in a row (the second with
a smaller list), on a graph kept in the caller's order and on a
degree-sorted one, plus the size limit."""
import numpy as np
import pytest
import torch  # (before the library's first call: one HIP runtime for both)

import paper_2604_22092_amd as fs
import workloads as W

pytestmark = pytest.mark.gpu

MODEL = {"ei": W.LN_E, "ir": W.LN_I, "beta": 0.15, "dt": 0.1, "seed": 29}
R = 4


def states(sim):
    return [sim.get_state(r) for r in range(R)]


def assert_same(a, b):
    for (sa, aa, ka), (sb, ab, kb) in zip(a, b):
        assert ka == kb
        np.testing.assert_array_equal(sa, sb)
        np.testing.assert_array_equal(aa, ab)


class NoAllocHook:
    """A device allocator that refuses every request and counts them."""

    def __init__(self):
        self.calls = 0

    def alloc(self, nbytes):
        self.calls += 1
        return 0

    def free(self, p):
        raise AssertionError("nothing was allocated")


@pytest.mark.parametrize("family", ["regular", "ba"])
@pytest.mark.parametrize("storage", [fs.FS_STORAGE_FP32, fs.FS_STORAGE_COMPACT])
def test_seed_noalloc_equals_seed(family, storage):
    if family == "regular":
        rp, ci = W.random_regular(20_000, 8, 3)      # identity order
    else:
        rp, ci = W.barabasi_albert(20_000, 4, 5)     # degree-sorted internal order
    n = len(rp) - 1
    rng = np.random.default_rng(7)
    # first call: 3000 ids (several staging pieces on the degree-sorted
    # graph), repeats included; second call: 17 ids into I of one replica
    first = rng.integers(0, n, 3000)
    second = rng.integers(0, n, 17)
    with fs.Graph(rp, ci) as g:
        a = fs.Sim.from_model(g, MODEL, steps_per_graph=10, replicas=R, storage=storage)
        b = fs.Sim.from_model(g, MODEL, steps_per_graph=10, replicas=R, storage=storage)
        try:
            for nodes, replica, comp in [(first, -1, fs.FS_E), (second, 1, fs.FS_I)]:
                a.seed(nodes, replica=replica, compartment=comp)
                hook = NoAllocHook()
                fs.set_allocator(hook.alloc, hook.free)
                try:
                    fs.fs_sim_seed_noalloc(b.handle, replica, nodes, comp)
                finally:
                    fs.set_allocator()
                assert hook.calls == 0
                assert_same(states(a), states(b))
                a.step(25)
                b.step(25)
                assert_same(states(a), states(b))
                k = a.step_index()
                for r in range(R):
                    np.testing.assert_array_equal(a.history(k - 25, 25, r), b.history(k - 25, 25, r))
        finally:
            a.close()
            b.close()


def test_seed_noalloc_size_limit():
    rp, ci = W.random_regular(70_000, 4, 1)
    n = len(rp) - 1
    with fs.Graph(rp, ci) as g:
        a = fs.Sim.from_model(g, MODEL, steps_per_graph=10, replicas=1)
        b = fs.Sim.from_model(g, MODEL, steps_per_graph=10, replicas=1)
        try:
            before = b.get_state(0)
            over = np.arange(fs.FS_SEED_NOALLOC_MAX + 1, dtype=np.int64) % n
            with pytest.raises(fs.FsError) as ei:
                fs.fs_sim_seed_noalloc(b.handle, 0, over, fs.FS_E)
            assert ei.value.status == 1 and str(fs.FS_SEED_NOALLOC_MAX) in str(ei.value)
            assert_same([before], [b.get_state(0)])
            # exactly the maximum is accepted
            full = over[:fs.FS_SEED_NOALLOC_MAX]
            a.seed(full, replica=0)
            fs.fs_sim_seed_noalloc(b.handle, 0, full, fs.FS_E)
            assert_same([a.get_state(0)], [b.get_state(0)])
        finally:
            a.close()
            b.close()
