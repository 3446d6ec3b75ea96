"""Seeded request mix for the scenario server: a pool of contact graphs and a
Poisson stream of scenario solves drawn over it.

Graph pool: N = round(exp(U(ln 1e4, ln 2e6))) (rounded to even), family
uniform over random k-regular (k uniform in 4..16, built as a union of k
random perfect matchings), Erdos-Renyi with mean degree 10, and
Barabasi-Albert with m uniform in 2..8.

Requests arrive as a Poisson process; each picks a pool graph uniformly, its
E->I and I->R laws uniformly among log-normal (mu of ln tau in U[ln 2, ln 6],
sigma in U[0.3, 0.8]), Weibull (shape U[1.5, 3], scale U[3, 8] d) and
Erlang (k uniform in 2..5, mean U[2, 6] d), beta in U[0.02, 0.1], dt = 0.1 d,
16 replicas, 300 steps, a fresh Philox seed, and max(10, N/1000) initially
exposed nodes.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import math

import numpy as np

from .graphs import barabasi_albert, erdos_renyi, random_regular_matchings

FAMILIES = ("regular", "er", "ba")


def pool_specs(size: int, seed: int, n_min: float = 1e4, n_max: float = 2e6):
    """Graph specs of the pool: (family, n, parameter, graph seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(size):
        fam = FAMILIES[i % 3] if size >= 3 else FAMILIES[int(rng.integers(0, 3))]
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) / 2)) * 2
        if fam == "regular":
            par = int(rng.integers(4, 17))
        elif fam == "er":
            par = 10.0
        else:
            par = int(rng.integers(2, 9))
        out.append((fam, n, par, int(rng.integers(0, 2**31))))
    return out


def build_graph(spec):
    fam, n, par, s = spec
    if fam == "regular":
        return random_regular_matchings(n, par, s)
    if fam == "er":
        return erdos_renyi(n, par, s)
    return barabasi_albert(n, par, s)


def _law(rng):
    kind = int(rng.integers(0, 3))
    if kind == 0:
        return ("lognormal", float(rng.uniform(math.log(2.0), math.log(6.0))), float(rng.uniform(0.3, 0.8)))
    if kind == 1:
        return ("weibull", float(rng.uniform(1.5, 3.0)), float(rng.uniform(3.0, 8.0)))
    k = int(rng.integers(2, 6))
    mean = float(rng.uniform(2.0, 6.0))
    return ("erlang", k, k / mean)


def requests(count: int, rate: float, pool_sizes, seed: int, replicas: int = 16, steps: int = 300,
             dt: float = 0.1):
    """`count` requests with Poisson arrival times (seconds from 0) over a
    pool whose graphs have the node counts `pool_sizes`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        gi = int(rng.integers(0, len(pool_sizes)))
        n = int(pool_sizes[gi])
        nseed = max(10, n // 1000)
        out.append({
            "arrival": t, "graph": gi, "ei": _law(rng), "ir": _law(rng),
            "beta": float(rng.uniform(0.02, 0.1)), "dt": dt, "seed": int(rng.integers(0, 2**63)),
            "replicas": replicas, "steps": steps,
            "seeds": np.sort(rng.choice(n, size=nseed, replace=False)).astype(np.int64),
        })
    return out
