"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle sources are compiled a second time, with -fsanitize=address,
undefined (host code only: gcc, no device code is involved), into a
separate library, and a child Python process drives every exported entry
point on small inputs, edge cases included: a one-node graph, empty rows,
self-loops and repeated edges, weights, both age storages, every holding-
time law, shedding profiles, the adaptive step rule, the exact simulator and
the Markovian engine.  Any out-of-bounds access, use of freed memory,
signed overflow, misaligned load or invalid shift aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import numpy as np
import oracle
import workloads as W

LAWS = [W.LN_E, ("weibull", 2.0, 6.0), ("weibull", 1.0, 3.0), ("erlang", 3, 1.0), ("erlang", 1, 0.5),
        ("exp", 0.3), ("lognormal", 1.2, 0.5)]
oracle.philox4x32(np.arange(64, dtype=np.uint32).reshape(16, 4), [1, 2])
oracle.philox4x64(np.arange(64, dtype=np.uint64).reshape(16, 4), [3, 4])
oracle.uniforms(2**40 + 5, np.arange(100), 7, 3)
oracle.erfcx(np.linspace(-30.0, 1e6, 4001))
tau = np.concatenate([[0.0, 1e-30, 1e-12], np.linspace(0.0, 500.0, 2001)])
for law in LAWS:
    oracle.hazard(law, tau)
    oracle.density(law, tau)

graphs = [
    (np.array([0, 0]), np.array([], np.int32)),                   # one node, no edge
    (np.array([0, 1]), np.array([0])),                            # one node, self-loop
    (np.array([0, 2, 2, 5]), np.array([1, 1, 0, 1, 2])),          # empty row, repeated edge
    W.random_regular(200, 6, 1),
    W.barabasi_albert(300, 3, 2),
]
rng = np.random.default_rng(0)
for rp, ci in graphs:
    n = len(rp) - 1
    w = rng.random(len(ci)).astype(np.float32)
    st = rng.integers(0, 4, n).astype(np.int32)
    for compact in (False, True):
        age = rng.integers(0, 300, n).astype(np.uint16) if compact else (rng.random(n) * 30).astype(np.float32)
        for ei, ir in zip(LAWS, LAWS[1:] + LAWS[:1]):
            for shed in (None, ("density", W.LN_I, 2.0), ("hazard", ("weibull", 2.0, 6.0), 1.0)):
                model = {"ei": ei, "ir": ir, "beta": 0.3, "dt": 0.1, "seed": 11, "shed": shed}
                for graph in ((rp, ci), (rp, ci, w)):
                    iota = oracle.infectivity(model, st, age, compact)
                    oracle.step(graph, model, st, age, iota, 5, replica=2, compact=compact)
                    oracle.step_nodes(graph, model, st, age, iota, 5, np.arange(n)[::2], compact=compact)
                    oracle.run(graph, model, st, age, 4, step0=3, compact=compact)
                if not compact:
                    oracle.run_adaptive((rp, ci), model, st, age, 4, 0.03, 0.1)
    oracle.next_dt(0.0, 0.03, 0.1)
    if n > 1:
        init = np.zeros(n, np.int32)
        init[0] = 1
        oracle.gillespie((rp, ci), W.LN_E, W.LN_I, 0.4, 30.0, init, 3, 4)
        oracle.gillespie((rp, ci, w), ("exp", 0.5), ("erlang", 2, 1.0), 0.4, 30.0, init, 4, 2)
    for mm in ("seir", "sir", "sis"):
        m = {"model": mm, "beta": 0.3, "sigma": 0.2, "gamma": 0.15, "theta": 0.01, "p_max": 0.1,
             "tau_max": 1.0, "seed": 2}
        st0 = rng.integers(0, 3, n).astype(np.int32)
        oracle.markov_tau((rp, ci), m, st0)
        oracle.markov_step((rp, ci), m, st0, 4)
        oracle.markov_run((rp, ci), m, st0, 6, k0=2)
print("sanitized oracle ok")
'''


def test_oracle_under_address_and_undefined_behavior_sanitizers(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    import oracle
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=c11", "-Wall",
                    "-o", lib, *oracle.SOURCES, "-lm"], check=True)
    env = dict(os.environ, FS_ORACLE_LIB=lib, LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    res = subprocess.run([sys.executable, "-c", DRIVER], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=600)
    report = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, report
    assert "sanitized oracle ok" in res.stdout, report
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, report
