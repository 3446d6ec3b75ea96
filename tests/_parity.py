"""Comparison rules between the HIP step and the FP64 oracle.

One step from an identical state must give identical per-node states, except
draws whose uniform lies within GUARD of the FP64 threshold q (a 1-ulp
difference in FP32 q can flip those); each such case is logged and their
number must stay strictly below 1e-6 of the node-updates compared (so none is
tolerated in a comparison of at most 1e6 updates).  Where states agree, ages
are bit-identical.  Rates agree with the FP64 rates to RATE_TOL relative
(the hazard tolerance), wherever the FP64 rate is inside the FP32 normal
range with margin (>= 1e-30); below it the FP32 rate must be tiny too.
"""
import numpy as np

GUARD = 1e-6
RATE_TOL = 2e-6
RATE_FLOOR = 1e-30


def guard_band_mismatches(gpu_state, ora_state, ora_u, ora_q, label=""):
    mism = np.flatnonzero(np.asarray(gpu_state) != np.asarray(ora_state))
    bad = []
    for i in mism:
        u, q = float(ora_u[i]), float(ora_q[i])
        if u >= 0.0 and abs(u - q) < GUARD:
            print(f"[guard band] {label} node {i}: u={u!r} q64={q!r} "
                  f"gpu={int(gpu_state[i])} oracle={int(ora_state[i])}")
        else:
            bad.append((int(i), u, q, int(gpu_state[i]), int(ora_state[i])))
    assert not bad, f"{label}: {len(bad)} state mismatches outside the guard band, first {bad[:5]}"
    return len(mism)


def check_mismatch_budget(n_mismatch, n_updates, label=""):
    assert n_mismatch == 0 or n_mismatch < 1e-6 * n_updates, \
        f"{label}: {n_mismatch} guard-band flips in {n_updates} updates"


def check_rates(gpu_rates, ora_lam, label=""):
    g = np.asarray(gpu_rates, dtype=np.float64)
    o = np.asarray(ora_lam, dtype=np.float64)
    assert not np.isnan(g).any(), f"{label}: NaN rates at {np.flatnonzero(np.isnan(g))[:5]}"
    big = o >= RATE_FLOOR
    rel = np.abs(g[big] - o[big]) / o[big]
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= RATE_TOL, f"{label}: rate relative error {worst:.3e} > {RATE_TOL}"
    small = ~big
    off = np.flatnonzero(small)[np.abs(g[small]) > 1e-29]
    assert off.size == 0, f"{label}: tiny rates not tiny on GPU at {off[:5]}: {g[off[:5]]} vs {o[off[:5]]}"
    return worst


def check_one_step(gpu, ora, prev_state, label=""):
    """gpu: dict(state, age, rates); ora: oracle.step output."""
    n = len(prev_state)
    nm = guard_band_mismatches(gpu["state"], ora["state"], ora["u"], ora["q"], label)
    check_mismatch_budget(nm, n, label)
    same = np.asarray(gpu["state"]) == np.asarray(ora["state"])
    np.testing.assert_array_equal(np.asarray(gpu["age"])[same], np.asarray(ora["age"])[same],
                                  err_msg=f"{label}: ages differ")
    worst = None
    if gpu.get("rates") is not None:
        worst = check_rates(gpu["rates"], ora["lam"], label)
    return nm, worst
