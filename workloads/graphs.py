"""Seeded random contact graphs as incoming-edge CSR arrays (int32).

Undirected graphs are returned symmetric: edge {u, v} appears as v in row u and
as u in row v.  Columns are sorted within each row.  All generators are
deterministic functions of their arguments (numpy PCG64 streams).
"""
from __future__ import annotations

import numpy as np


def csr_from_edges(n: int, src, dst, symmetric: bool = True):
    """CSR of row = dst (the node that receives), col = src.

    With symmetric=True each undirected pair (src[i], dst[i]) contributes both
    directions.  Duplicates are kept (they count with multiplicity).
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if symmetric:
        rows = np.concatenate([src, dst])
        cols = np.concatenate([dst, src])
    else:
        rows, cols = dst, src
    key = rows * np.int64(n) + cols
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("edge count does not fit int32")
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def _bad_edges(u, v, n):
    """Indices of self-loops and of every repeat of an already-seen pair."""
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * np.int64(n) + b
    order = np.argsort(key, kind="stable")
    ks = key[order]
    dup = np.zeros(len(u), dtype=bool)
    dup[order[1:][ks[1:] == ks[:-1]]] = True
    return np.flatnonzero(dup | (u == v))


def random_regular(n: int, d: int, seed: int):
    """Random simple d-regular graph: configuration model, then random
    degree-preserving double-edge swaps until no self-loop or multi-edge is
    left (rejection is hopeless at d = 10: a simple pairing occurs with
    probability about exp(-(d^2-1)/4))."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    u = stubs[0::2].copy()
    v = stubs[1::2].copy()
    del stubs
    m = len(u)
    for _ in range(1000):
        bad = _bad_edges(u, v, n)
        if len(bad) == 0:
            break
        partners = rng.integers(0, m, size=len(bad))
        flips = rng.random(len(bad)) < 0.5
        used = set()
        for e, f, flip in zip(bad.tolist(), partners.tolist(), flips.tolist()):
            if e == f or e in used or f in used:
                continue
            used.add(e)
            used.add(f)
            a, b, c, dd = u[e], v[e], u[f], v[f]
            # {a,b},{c,dd} -> {a,c},{b,dd}  or  {a,dd},{b,c}: degrees preserved
            if flip:
                u[e], v[e], u[f], v[f] = a, c, b, dd
            else:
                u[e], v[e], u[f], v[f] = a, dd, b, c
    else:
        raise RuntimeError("double-edge swap repair did not converge")
    return csr_from_edges(n, u, v, symmetric=True)


def _batcher_pairs(k: int):
    """Comparators (i, j), i < j, of Batcher's odd-even merge sort for k keys
    (the network for the next power of two with every comparator that touches
    a key >= k dropped, which is still a sorting network for k keys)."""
    pairs = []
    p = 1
    while p < k:
        q = p
        while q >= 1:
            r = q % p
            for jj in range(r, k - q, 2 * q):
                for i in range(min(q, k - jj - q)):
                    if (i + jj) // (2 * p) == (i + jj + q) // (2 * p):
                        pairs.append((i + jj, i + jj + q))
            q //= 2
        p *= 2
    return pairs


def random_regular_matchings(n: int, d: int, seed: int):
    """Random simple d-regular graph as the union of d independent uniform
    perfect matchings (n even), for sizes where the configuration model's
    sort-based repair is too slow (N = 1e8).  For d >= 3 this law is contiguous
    to the uniform random d-regular graph (Molloy, Robalewska, Robinson and
    Wormald, 1997), so the two agree on every property that holds with high
    probability.

    Matching m pairs perm_m[2i] with perm_m[2i+1] for a uniform permutation
    perm_m, and P[m, a] is the partner of a in it.  The row of node a is
    [P[0, a], ..., P[d-1, a]], so the CSR is written directly (row_ptr = d a).
    A pair repeated across two matchings (about d(d-1)/4 of them in
    expectation, independent of n) is removed by a swap inside the later
    matching: {a,b},{c,e} -> {a,c},{b,e}, which keeps it a perfect matching and
    every degree at d.  Rows are returned sorted.
    """
    if n % 2:
        raise ValueError("n must be even")
    if 2 * d > n:
        raise ValueError("the matching union is for sparse graphs: need 2 d <= n")
    if n * d >= 2**31:
        raise ValueError("edge count does not fit int32")
    rng = np.random.default_rng(seed)
    P = np.empty((d, n), dtype=np.int32)
    for m in range(d):
        perm = rng.permutation(n).astype(np.int32)
        P[m, perm[0::2]] = perm[1::2]
        P[m, perm[1::2]] = perm[0::2]
        del perm
    for _ in range(200):
        bad = np.zeros(n, dtype=bool)
        for m in range(1, d):
            for m0 in range(m):
                bad |= P[m] == P[m0]
        bad = np.flatnonzero(bad)
        if len(bad) == 0:
            break
        done = set()
        for a in bad.tolist():
            row = P[:, a].tolist()
            for m in range(1, d):
                b = row[m]
                if b in row[:m] and a not in done and b not in done:
                    # move the later copy of {a, b}: swap with a random edge {c, e}
                    # of matching m (a later round retries if no partner is found)
                    for _try in range(64):
                        c = int(rng.integers(0, n))
                        e = int(P[m, c])
                        if (len({a, b, c, e}) == 4 and c not in P[:, a].tolist()
                                and e not in P[:, b].tolist()):
                            P[m, a], P[m, c] = c, a
                            P[m, b], P[m, e] = e, b
                            done.update((a, b, c, e))
                            break
                    break
    else:
        raise RuntimeError("matching repair did not converge")
    tmp = np.empty(n, dtype=np.int32)
    for i, j in _batcher_pairs(d):
        np.minimum(P[i], P[j], out=tmp)
        np.maximum(P[i], P[j], out=P[j])
        P[i] = tmp
    del tmp
    col = np.ascontiguousarray(P.T).reshape(-1)
    del P
    return np.arange(0, (n + 1) * d, d, dtype=np.int32), col


def erdos_renyi(n: int, mean_degree: float, seed: int):
    """G(n, p) with p = mean_degree/(n-1): the edge count is Binomial(n(n-1)/2, p)
    and, given the count, the edge set is a uniform set of distinct pairs."""
    rng = np.random.default_rng(seed)
    pairs = n * (n - 1) // 2
    p = mean_degree / (n - 1)
    m = int(rng.binomial(pairs, p))
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < m:
        need = m - len(keys)
        a = rng.integers(0, n, size=int(need * 1.1) + 16, dtype=np.int64)
        b = rng.integers(0, n, size=len(a), dtype=np.int64)
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        keys = np.unique(np.concatenate([keys, lo * n + hi]))
    if len(keys) > m:
        keys = rng.choice(keys, size=m, replace=False)
    return csr_from_edges(n, keys // n, keys % n, symmetric=True)


def barabasi_albert(n: int, m: int, seed: int):
    """Barabasi-Albert preferential attachment in the repeated-endpoint-list form
    of Batagelj & Brandes (2005), started from the complete graph K_{m+1}.

    Each new node v >= m+1 adds m edges; the far endpoint of each is a uniform
    pick from the list of all endpoints placed so far (so proportional to
    degree).  The list is resolved with vectorised pointer jumping.  Self-loops
    and repeated pairs that the sampling produces are dropped, so the graph is
    simple (mean degree slightly below 2m).
    """
    if n <= m + 1:
        return complete_graph(n)
    rng = np.random.default_rng(seed)
    # endpoint list of the initial clique
    cu, cv = np.triu_indices(m + 1, k=1)
    base_list = np.empty(2 * len(cu), dtype=np.int64)
    base_list[0::2] = cu
    base_list[1::2] = cv
    base = len(base_list)
    new_nodes = n - (m + 1)
    j = np.arange(new_nodes * m, dtype=np.int64)      # edge index of the appended slots
    owner = (m + 1) + j // m                            # node that adds edge j
    # slot of edge j's own endpoint: base + 2j; far endpoint: base + 2j + 1 chosen
    # uniformly from the slots filled before it, [0, base + 2j + 1)
    bound = base + 2 * j + 1
    r = np.floor(rng.random(len(j)) * bound).astype(np.int64)
    r = np.minimum(r, bound - 1)
    target = np.empty(len(j), dtype=np.int64)
    unresolved = np.arange(len(j), dtype=np.int64)
    ptr = r.copy()
    while len(unresolved):
        p = ptr[unresolved]
        in_base = p < base
        off = p - base
        even = (~in_base) & (off % 2 == 0)
        odd = (~in_base) & (off % 2 == 1)
        target[unresolved[in_base]] = base_list[p[in_base]]
        target[unresolved[even]] = (m + 1) + (off[even] // 2) // m
        # an odd slot holds the far endpoint of an earlier edge: follow its pick
        ptr[unresolved[odd]] = r[(off[odd] - 1) // 2]
        unresolved = unresolved[odd]
    src = np.concatenate([cu.astype(np.int64), owner])
    dst = np.concatenate([cv.astype(np.int64), target])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    keys = np.unique(lo * n + hi)
    return csr_from_edges(n, keys // n, keys % n, symmetric=True)


def complete_graph(n: int):
    """K_n: every node receives from every other node."""
    a, b = np.triu_indices(n, k=1)
    return csr_from_edges(n, a, b, symmetric=True)


def star_forest(n_stars: int, leaves: int):
    """n_stars disjoint stars; star s has centre s*(leaves+1) and `leaves`
    leaves that point INTO the centre only (directed: row centre lists the
    leaves, leaf rows are empty)."""
    centres = np.arange(n_stars, dtype=np.int64) * (leaves + 1)
    src = (centres[:, None] + 1 + np.arange(leaves)[None, :]).ravel()
    dst = np.repeat(centres, leaves)
    return csr_from_edges(n_stars * (leaves + 1), src, dst, symmetric=False)


def paper_csr_example():
    """The five-node incoming-edge CSR printed in the paper's data-layout appendix
    (figure of the CSR layout): row_ptr [0,2,3,6,8,9], col_ind [1,3,0,1,3,4,0,2,1].
    It is a valid CSR but not symmetric (row 1 lists only node 0)."""
    return (np.array([0, 2, 3, 6, 8, 9], dtype=np.int32),
            np.array([1, 3, 0, 1, 3, 4, 0, 2, 1], dtype=np.int32))
