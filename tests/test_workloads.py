"""Input generators: the graphs have the structure their families promise.

These generators feed both the oracle and the HIP path; the checks here are
on graph structure only (degrees, symmetry, simplicity, determinism).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from workloads.graphs import _batcher_pairs


def simple_symmetric(rp, ci):
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert not (rows == ci).any(), "self-loop"
    for i in range(0, n, max(1, n // 2000)):
        r = ci[rp[i]:rp[i + 1]]
        assert (np.diff(r) > 0).all(), f"row {i} unsorted or repeated"
    a = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    assert (a != a.T).nnz == 0, "not symmetric"


@pytest.mark.parametrize("k", range(1, 17))
def test_batcher_network_sorts_all_binary_inputs(k):
    # 0-1 principle: a comparator network that sorts every 0/1 vector sorts everything
    pairs = _batcher_pairs(k)
    v = (np.arange(1 << k)[:, None] >> np.arange(k)[None, :]) & 1
    for i, j in pairs:
        lo = np.minimum(v[:, i], v[:, j])
        v[:, j] = np.maximum(v[:, i], v[:, j])
        v[:, i] = lo
    assert (np.diff(v, axis=1) >= 0).all()


@pytest.mark.parametrize("n,d", [(10, 3), (12, 6), (1000, 8), (20_000, 16), (200_000, 8)])
def test_matching_union_is_simple_regular(n, d):
    rp, ci = W.random_regular_matchings(n, d, 3)
    assert rp.dtype == np.int32 and ci.dtype == np.int32
    np.testing.assert_array_equal(np.diff(rp), d)
    simple_symmetric(rp, ci)
    rp2, ci2 = W.random_regular_matchings(n, d, 3)
    np.testing.assert_array_equal(ci, ci2)
    _, ci3 = W.random_regular_matchings(n, d, 4)
    assert not np.array_equal(ci, ci3)


def test_matching_union_edges_are_uniform_pairs():
    # every node's neighbours are spread over the whole id range (a matching
    # pairs uniform random nodes): the mean neighbour id is near (n-1)/2
    n, d = 100_000, 8
    _, ci = W.random_regular_matchings(n, d, 5)
    m = ci.reshape(n, d).mean(1)
    assert abs(m.mean() / (n - 1) - 0.5) < 0.002


def test_matching_union_rejects_bad_sizes():
    with pytest.raises(ValueError):
        W.random_regular_matchings(11, 3, 0)
    with pytest.raises(ValueError):
        W.random_regular_matchings(8, 5, 0)


@pytest.mark.parametrize("gen", ["regular", "er", "ba"])
def test_other_families_simple(gen):
    if gen == "regular":
        rp, ci = W.random_regular(5000, 10, 0)
        np.testing.assert_array_equal(np.diff(rp), 10)
    elif gen == "er":
        rp, ci = W.erdos_renyi(20_000, 10.0, 0)
        assert abs(len(ci) / 20_000 - 10.0) < 0.3
    else:
        rp, ci = W.barabasi_albert(20_000, 5, 0)
        deg = np.diff(rp)
        assert deg.min() >= 1 and deg.max() > 100  # heavy tail
        assert 9.0 < deg.mean() <= 10.0
    simple_symmetric(rp, ci)
