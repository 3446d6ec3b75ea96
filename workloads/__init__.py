"""Seeded synthetic inputs for the renewal tau-leap step.

This module serves both the HIP library's tests/benchmark and the CPU oracle.
It holds none of the method's arithmetic: only graph generators (incoming-edge
CSR, symmetric for undirected graphs), seed-node selection and the named
workload descriptions.  The paper benchmarks only synthetic random graphs
(Erdos-Renyi, Barabasi-Albert, fixed degree); these generators produce graphs
of the same families and sizes.

A model description is a plain dict:
    {"ei": law, "ir": law, "beta": float, "dt": float, "seed": int}
with holding-time laws as tuples ("lognormal", mu, sigma), ("weibull", shape,
scale), ("erlang", k, rate) or ("exp", rate).
"""
from __future__ import annotations

import math

import numpy as np

from .graphs import (barabasi_albert, complete_graph, csr_from_edges, erdos_renyi,
                     paper_csr_example, random_regular, random_regular_matchings, star_forest)

__all__ = ["barabasi_albert", "complete_graph", "csr_from_edges", "erdos_renyi",
           "paper_csr_example", "random_regular", "random_regular_matchings", "star_forest", "seed_nodes",
           "initial_state", "WORKLOADS", "workload_graph", "LN_E", "LN_I"]

# Log-normal holding times of the plain SEIR workloads: E ~ LN(ln 3, 0.5),
# I ~ LN(ln 5, 0.6), parameters of ln(tau) in days.
LN_E = ("lognormal", math.log(3.0), 0.5)
LN_I = ("lognormal", math.log(5.0), 0.6)


def seed_nodes(n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct node ids drawn uniformly (numpy PCG64 seeded with `seed`)."""
    rng = np.random.default_rng(seed)
    count = min(int(count), int(n))
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def initial_state(n: int, seeds, compartment: int = 1) -> np.ndarray:
    """All nodes susceptible (0) except `seeds`, placed in `compartment` (E = 1)."""
    st = np.zeros(n, dtype=np.int32)
    st[np.asarray(seeds, dtype=np.int64)] = compartment
    return st


# Named workloads (synthetic graphs of the paper's families).  "steps" is the
# trajectory length; "seeds" the number of initially exposed nodes.
WORKLOADS = {
    # random 10-regular graph, N = 1e4: the small parity case
    "regular10_n1e4": {
        "graph": ("regular", 10_000, 10, 0),
        "model": {"ei": LN_E, "ir": LN_I, "beta": 0.06, "dt": 0.1, "seed": 0},
        "steps": 300, "seeds": 10, "seed_rng": 100, "storage": "fp32",
    },
    # random 10-regular graph, N = 1e6, single replica, captured step loop
    "regular10_n1e6": {
        "graph": ("regular", 1_000_000, 10, 1),
        "model": {"ei": LN_E, "ir": LN_I, "beta": 0.06, "dt": 0.1, "seed": 0},
        "steps": 500, "seeds": 100, "seed_rng": 101, "storage": "fp32",
    },
    # Barabasi-Albert, N = 1e6, m = 5; Erlang(k=3, mean 3 d) and Weibull(2, 6 d)
    "ba5_n1e6": {
        "graph": ("ba", 1_000_000, 5, 2),
        "model": {"ei": ("erlang", 3, 1.0), "ir": ("weibull", 2.0, 6.0), "beta": 0.03,
                  "dt": 0.1, "seed": 0},
        "steps": 500, "seeds": 100, "seed_rng": 102, "storage": "fp32",
    },
    # random 8-regular graph, N = 1e8 (col_ind 3.2 GB), compact vs FP32 storage;
    # built as a union of 8 random perfect matchings (the configuration model's
    # sort-based repair does not scale to 8e8 stubs)
    "regular8_n1e8": {
        "graph": ("regular_m", 100_000_000, 8, 3),
        "model": {"ei": LN_E, "ir": LN_I, "beta": 0.07, "dt": 0.2, "seed": 0},
        "steps": 200, "seeds": 1000, "seed_rng": 103, "storage": "compact",
    },
}


def workload_graph(spec):
    """Build the CSR (row_ptr, col_ind) of a workload's graph tuple."""
    fam = spec[0]
    if fam == "regular":
        _, n, d, s = spec
        return random_regular(n, d, s)
    if fam == "regular_m":
        _, n, d, s = spec
        return random_regular_matchings(n, d, s)
    if fam == "ba":
        _, n, m, s = spec
        return barabasi_albert(n, m, s)
    if fam == "er":
        _, n, c, s = spec
        return erdos_renyi(n, c, s)
    raise ValueError(f"unknown graph family {fam!r}")
