"""Pins for the oracle's counter-based generator (Philox, Salmon et al. SC'11).

The method draws u from Philox4x32-10 keyed by (seed, replica, step, node).
The oracle's implementation is checked against two independent library
implementations:
  * numpy's Philox bit generator (the 4x64-10 instance of the same round
    function and key schedule) — pins the round structure, word order and
    key bumping;
  * rocRAND's Philox4x32-10 engine evaluated on the host — pins the 32-bit
    multipliers and Weyl constants and the exact counter/key layout.
Statistical checks (chi-square uniformity, per-bit balance) cover the
24-bit uniform conversion.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox4x64_matches_numpy(orc):
    rng = np.random.default_rng(7)
    total = 0
    for trial in range(40):
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        start = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        start[0] = np.uint64(rng.integers(0, 2**63))  # room to count up without wrap
        bg = np.random.Philox(key=key)
        st = bg.state
        st["state"]["counter"] = start.copy()
        bg.state = st
        blocks = 500
        raw = bg.random_raw(4 * blocks).reshape(blocks, 4)
        # numpy increments the 256-bit counter before generating each block
        ctr = np.tile(start, (blocks, 1))
        ctr[:, 0] = start[0] + np.arange(1, blocks + 1, dtype=np.uint64)
        mine = orc.philox4x64(ctr, key)
        np.testing.assert_array_equal(mine, raw)
        total += blocks
    assert total == 20000


def test_philox4x64_counter_carry_matches_numpy(orc):
    # word-0 overflow carries into word 1 inside numpy; the oracle maps a full counter
    key = np.array([3, 5], dtype=np.uint64)
    start = np.array([2**64 - 3, 11, 0, 0], dtype=np.uint64)
    bg = np.random.Philox(key=key)
    st = bg.state
    st["state"]["counter"] = start.copy()
    bg.state = st
    raw = bg.random_raw(4 * 6).reshape(6, 4)
    ctr = []
    c0, c1 = 2**64 - 3, 11
    for _ in range(6):
        c0 += 1
        if c0 == 2**64:
            c0, c1 = 0, c1 + 1
        ctr.append([c0, c1, 0, 0])
    np.testing.assert_array_equal(orc.philox4x64(np.array(ctr, dtype=np.uint64), key), raw)


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available for the host-side pin")
    d = tmp_path_factory.mktemp("rocrand_pin")
    exe = str(d / "rocrand_philox")
    subprocess.run([hipcc, "-O2", "-o", exe, os.path.join(HERE, "pins", "rocrand_philox.cpp")],
                   check=True, capture_output=True)
    return exe, d


def _rocrand_eval(pin, seed, ctr):
    exe, d = pin
    req = d / "req.bin"
    out = d / "out.bin"
    with open(req, "wb") as f:
        f.write(np.array([seed, len(ctr)], dtype=np.uint64).tobytes())
        f.write(np.ascontiguousarray(ctr, dtype=np.uint32).tobytes())
    subprocess.run([exe, str(req), str(out)], check=True)
    return np.fromfile(out, dtype=np.uint32).reshape(-1, 4)


def test_philox4x32_matches_rocrand(orc, rocrand_pin):
    rng = np.random.default_rng(11)
    n_total = 0
    for seed in [0, 1, 0x1234567887654321, int(rng.integers(0, 2**63))]:
        n = 250_000
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = rng.integers(0, 2**32, size=n, dtype=np.uint32)      # node
        ctr[:, 1] = rng.integers(0, 2**30, size=n, dtype=np.uint32)      # step
        ctr[:, 2] = rng.integers(0, 64, size=n, dtype=np.uint32)         # replica
        ctr[:100, 1] = np.arange(100)                                     # small steps too
        ctr[-100:, 3] = rng.integers(0, 2**32, size=100, dtype=np.uint32)
        key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
        ref = _rocrand_eval(rocrand_pin, seed, ctr)
        np.testing.assert_array_equal(orc.philox4x32(ctr, key), ref)
        n_total += n
    assert n_total >= 1_000_000


def test_uniform_grid_and_strict_range(orc):
    u = orc.uniforms(0, np.arange(200_000), step=3, replica=0)
    assert u.min() >= 0.0 and u.max() <= 1.0 - 2.0**-24
    # every value lies on the 2^-24 grid
    np.testing.assert_array_equal(u * 2**24, np.floor(u * 2**24))


def test_uniform_chi_square_and_bit_balance(orc):
    n = 400_000
    seed = 0xDEADBEEF12345
    u = np.concatenate([orc.uniforms(seed, np.arange(n // 4), step=s, replica=r)
                        for s, r in [(0, 0), (1, 0), (0, 1), (123456, 7)]])
    counts, _ = np.histogram(u, bins=256, range=(0.0, 1.0))
    chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
    # p-value bounds for 255 degrees of freedom, two-sided 1e-6
    assert stats.chi2.sf(chi2, 255) > 1e-6 and stats.chi2.cdf(chi2, 255) > 1e-6
    bits = (u * 2**24).astype(np.uint32)
    for b in range(24):
        ones = int(((bits >> b) & 1).sum())
        z = (ones - n / 2) / np.sqrt(n / 4)
        assert abs(z) < 5.5, (b, z)


def test_keying_distinguishes_node_step_replica_seed(orc):
    base = orc.uniforms(5, np.arange(1000), step=10, replica=2)
    for other in [orc.uniforms(6, np.arange(1000), 10, 2), orc.uniforms(5, np.arange(1000), 11, 2),
                  orc.uniforms(5, np.arange(1000), 10, 3), orc.uniforms(5, np.arange(1, 1001), 10, 2)]:
        assert np.mean(base == other) < 0.01
