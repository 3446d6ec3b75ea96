"""Throughput of the HIP renewal tau-leap step on one MI355X.

Workload: a seeded random 10-regular graph with N = 1e6 (configuration model
with double-edge-swap repair), SEIR with log-normal E (mu = ln 3, sigma = 0.5)
and I (mu = ln 5, sigma = 0.6) holding times, beta = 0.06 per edge per day,
dt = 0.1 d, 100 initially exposed nodes, FP32 storage, one replica, a
captured hipGraph of b steps per replay (b = 50, or K rounded down to even
when K < 50).  A step is one fused launch over all N nodes.  The configured
trajectory is 500 steps (50 days); it is run from the seeded start as timed
windows of exactly K steps (K = --steps, default the whole trajectory), each
bracketed by device synchronisations, so a short K still measures every
phase of the epidemic.  Inputs are resident in HBM throughout.

Prints one JSON line: GNUPS (node-updates per second / 1e9), the roofline
record of the step kernel (algorithmic bytes per launch over the measured
per-launch time against the 8 TB/s HBM peak, plus the counter-measured
traffic of the committed profile when it matches the kernel sources), the
FP64 oracle timed on the host (on one core, and as independent replicas on
every usable core), and a short sample of the scenario server (--serving
below) at 50 requests/s and at saturation.

--workload selects another named workload of the same kind (the
Barabasi-Albert graph with autotuned degree bins, or the N = 1e8 8-regular
graph with compact or FP32 storage); the default line is the one above.

--shed runs the same workload with an age-dependent shedding profile s(tau)
(Eq. (infectivity)): "hazard" is s = h_IR(tau), the form the paper's overhead
study writes in-kernel; "density" a log-normal shedding curve (median 2.5 d,
sigma 0.5) scaled to 5 infectious days; "unit" the profile s = 1 through the
shedding kernels (the constant run's trajectory, so its time against the
default line is the cost of the shedding path itself).  --compaction turns on active-node
compaction; --beta overrides the transmission rate (a saturating epidemic is
where compaction pays).

--markov measures the Markovian engine instead (Section "Markovian
engine"): SIR on an Erdos-Renyi graph with N = 1e6 and mean degree 8, beta =
0.25, gamma = 0.15, theta = 0.01, p_max = 0.1 (the paper's validation
model), 100 initially infectious nodes, captured replays of 50 steps, the
whole epidemic timed; it prints realized transitions per second, the
paper's measure for this engine, beside node-updates per second.

--serving measures the scenario server instead: a seeded Poisson stream of
scenario solves (16 replicas, 300 steps, graphs of 1e4..2e6 nodes from a
resident pool, laws and beta drawn per request) through the server, and the
same stream as sequential plain solves; it prints scenarios/s and p50/p99
latency (arrival to counts ready) for both.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GNUPS & % HBM roofline; batched-serving scenarios/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "regular10_n1e6"
GRAPH_TEXT = {
    "regular10_n1e6": "random 10-regular, N=1e6, configuration model, seed 1",
    "ba5_n1e6": "Barabasi-Albert m=5, N=1e6, seed 2",
    "regular8_n1e8": "random 8-regular, N=1e8, union of 8 random perfect matchings, seed 3",
}
LAW_TEXT = {
    "regular10_n1e6": "E~LN(ln3,0.5), I~LN(ln5,0.6)",
    "ba5_n1e6": "E~Erlang(3, rate 1), I~Weibull(2, 6)",
    "regular8_n1e8": "E~LN(ln3,0.5), I~LN(ln5,0.6)",
}
STEPS_PER_GRAPH = 50
SHEDS = {
    "none": None,
    "density": ("density", ("lognormal", 0.9162907318741551, 0.5), 5.0),   # median 2.5 d
    "unit": ("hazard", ("exp", 1.0), 1.0),
}


def bytes_per_update(d_mean: float, storage: str) -> float:
    """Algorithmic bytes per node-update: every per-node array moved once per
    step (state r/w, age r/w, row_ptr, next infectivity write, one unique
    infectivity read) plus the col_ind stream of the row (4 B per edge).
    FP32 storage: 28 + 4 d; compact: 14 + 4 d."""
    return (28.0 if storage == "fp32" else 14.0) + 4.0 * d_mean


STEP_KERNEL_SOURCES = ("fs_step.hpp", "fs_kernels.hip", "fs_device.hpp", "fs_internal.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources that define the step kernel (the counters of a
    committed profile stand only while it matches)."""
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_22092_amd", "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(rp, ci, model, seeds, budget_s: float, compact: bool):
    """The FP64 oracle (single thread) on the first steps of the same run."""
    import numpy as np

    import oracle
    import workloads as W

    n = len(rp) - 1
    st = W.initial_state(n, seeds)
    age = np.zeros(n, np.uint16 if compact else np.float32)
    per_call = max(1, min(5, int(2e7 // n)))
    st, age, _ = oracle.run((rp, ci), model, st, age, 1, compact=compact)  # load + first touch
    steps, t0 = 0, time.perf_counter()
    while True:
        st, age, _ = oracle.run((rp, ci), model, st, age, per_call, step0=1 + steps, compact=compact)
        steps += per_call
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": n * steps / el / 1e9, "unit": "GNUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps (steps 1..{steps}) of the same N={n:.0e} trajectory, "
                      f"single-threaded FP64 oracle, {el:.1f} s"}


def load_graph(spec, cache_dir=None):
    """The workload graph of `spec`, generated, or loaded from (and saved to)
    cache_dir as .npy files (the generators are deterministic in spec)."""
    import numpy as np

    import workloads as W
    if not cache_dir:
        return W.workload_graph(spec)
    os.makedirs(cache_dir, exist_ok=True)
    base = os.path.join(cache_dir, "graph_" + "_".join(str(x) for x in spec))
    if os.path.exists(base + "_ci.npy"):
        return np.load(base + "_rp.npy"), np.load(base + "_ci.npy")
    rp, ci = W.workload_graph(spec)
    np.save(base + "_rp.npy", rp)
    np.save(base + "_ci.npy", ci)
    return rp, ci


def host_cores() -> int:
    """Cores this process may use, capped at 16 (the host CPU share of one GPU on a shared node)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def cpu_all_cores(rp, ci, model, seeds, budget_s: float, compact: bool):
    """The host's embarrassingly parallel throughput: P independent replicas
    of the same run (replica ids 0..P-1, so independent Philox streams), one
    single-threaded FP64 oracle per core, P = the usable cores (at most 16,
    fewer when P copies of the state would not fit in 32 GB)."""
    import threading

    import numpy as np

    import oracle
    import workloads as W

    n = len(rp) - 1
    P = min(host_cores(), max(1, int(32e9 // (n * 40))))
    per_call = max(1, min(5, int(2e7 // n)))
    done = [0] * P
    errs = []
    t_end = [0.0]

    def worker(r):
        try:
            st = W.initial_state(n, seeds)
            age = np.zeros(n, np.uint16 if compact else np.float32)
            k = 0
            while time.perf_counter() < t_end[0]:
                st, age, _ = oracle.run((rp, ci), model, st, age, per_call, step0=k, replica=r,
                                        compact=compact)
                k += per_call
                done[r] = k
        except Exception as e:  # (reported, never hidden)
            errs.append(repr(e))

    oracle.lib()
    t0 = time.perf_counter()
    t_end[0] = t0 + budget_s
    ths = [threading.Thread(target=worker, args=(r,)) for r in range(P)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    if errs:
        raise RuntimeError(f"oracle worker failed: {errs[0]}")
    total = sum(done)
    return {"value": n * total / el / 1e9, "unit": "GNUPS", "cores": P, "kind": "oracle",
            "sample": f"{P} independent replicas of the same N={n:.0e} run from the seeded start, "
                      f"one single-threaded FP64 oracle per core ({min(done)}..{max(done)} steps each), "
                      f"{el:.1f} s"}


def copy_bandwidth(torch, dev, mib: int = 1024, reps: int = 5) -> float:
    """Measured device-to-device copy bandwidth (bytes read + written per
    second, GB/s): the best of `reps` copies of `mib` MiB."""
    src = torch.empty(mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2.0 * (mib << 20) / (best / 1e3) / 1e9


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def serving_run(n_req: int, rate: float, pool_size: int, slots: int = 0, round_steps: int = 0,
                label: str = "serving", graphs_cache=None):
    """The seeded request stream through the scenario server, and the same
    stream as sequential plain solves (each starting when it has arrived and
    the previous one is done).  rate = 0 offers every request at once
    (saturation).  Returns the record of both modes."""
    import threading

    import numpy as np

    import paper_2604_22092_amd as fs
    import workloads.serving as WS

    fs.lib()  # fail loudly without the HIP library
    t0 = time.perf_counter()
    if graphs_cache is not None and graphs_cache.get("size") == pool_size:
        graphs, sizes = graphs_cache["graphs"], graphs_cache["sizes"]
    else:
        specs = WS.pool_specs(pool_size, seed=404)
        pool = [WS.build_graph(sp) for sp in specs]
        sizes = [len(rp) - 1 for rp, _ in pool]
        graphs = [fs.Graph(rp, ci) for rp, ci in pool]
        del pool
        print(f"[{label}] pool of {len(graphs)} graphs (N {min(sizes)}..{max(sizes)}) built in "
              f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
        if graphs_cache is not None:
            graphs_cache.update(size=pool_size, graphs=graphs, sizes=sizes)
        # warm-up: every pool graph once (kernels loaded, the graphs' row
        # layouts for 16 replicas built and cached, as for resident graphs)
        for gi in range(len(graphs)):
            r = dict(WS.requests(1, 50.0, sizes, seed=405)[0], graph=gi, steps=4,
                     seeds=np.array([0, 1], np.int64))
            sim = fs.Sim(graphs[gi], r["ei"], r["ir"], r["beta"], r["dt"], seed=r["seed"], replicas=16)
            sim.seed(r["seeds"], replica=-1)
            sim.step(4)
            sim.counts(0)
            sim.close()
    reqs = WS.requests(n_req, rate if rate > 0 else 50.0, sizes, seed=405)
    if rate <= 0:
        for r in reqs:
            r["arrival"] = 0.0
    updates = sum(sizes[r["graph"]] * r["replicas"] * r["steps"] for r in reqs)
    span_offered = reqs[-1]["arrival"]

    def plain_solve(r):
        sim = fs.Sim(graphs[r["graph"]], r["ei"], r["ir"], r["beta"], r["dt"], seed=r["seed"],
                     replicas=r["replicas"], history_len=max(r["steps"], 2))
        sim.seed(r["seeds"], replica=-1)
        sim.step(r["steps"])
        h = np.stack([sim.history(0, r["steps"], k) for k in range(r["replicas"])], axis=1)
        sim.close()
        return h

    # batched: the server, with requests submitted at their arrival times
    sv = fs.Server(max_active=slots, steps_per_round=round_steps)
    ids = [None] * len(reqs)
    start = fs.fs_server_clock() + 0.05

    def submitter():
        for i, r in enumerate(reqs):
            delay = start + r["arrival"] - fs.fs_server_clock()
            if delay > 0:
                time.sleep(delay)
            ids[i] = sv.submit(graphs[r["graph"]], r["ei"], r["ir"], r["beta"], r["dt"], r["seed"],
                               r["replicas"], r["steps"], r["seeds"])

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    check = set(range(0, len(reqs), max(1, len(reqs) // 8)))
    b_hist, b_info = {}, []
    for i, rid in enumerate(ids):
        sv.wait(rid)
        h, info = sv.result(rid)
        b_info.append(info)
        if i in check:
            b_hist[i] = h
    sv.close()
    b_lat = [x["t_done"] - x["t_submit"] for x in b_info]
    b_span = max(x["t_done"] for x in b_info) - start
    print(f"[{label}] batched: {len(reqs) / b_span:.1f} scenarios/s, p50 {percentile(b_lat, 50):.3f}s "
          f"p99 {percentile(b_lat, 99):.3f}s", file=sys.stderr, flush=True)

    s_lat = []
    same = 0
    start = time.perf_counter() + 0.05
    for i, r in enumerate(reqs):
        delay = start + r["arrival"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        h = plain_solve(r)
        s_lat.append(time.perf_counter() - (start + r["arrival"]))
        if i in b_hist:
            if not np.array_equal(h, b_hist[i]):
                raise SystemExit(f"request {i}: batched and sequential counts differ")
            same += 1
    s_span = time.perf_counter() - start
    print(f"[{label}] sequential: {len(reqs) / s_span:.1f} scenarios/s, p50 {percentile(s_lat, 50):.3f}s "
          f"p99 {percentile(s_lat, 99):.3f}s", file=sys.stderr, flush=True)

    def rec(n, span, lat):
        return {"scenarios_per_s": round(n / span, 3), "p50_s": round(percentile(lat, 50), 4),
                "p99_s": round(percentile(lat, 99), 4), "makespan_s": round(span, 3),
                "gnups": round(updates / span / 1e9, 3)}

    return {"requests": len(reqs), "rate_per_s": rate if rate > 0 else "all at once",
            "pool_graphs": len(graphs), "n_range": [min(sizes), max(sizes)],
            "batched": rec(len(reqs), b_span, b_lat), "sequential": rec(len(reqs), s_span, s_lat),
            "identical_counts_checked": same,
            "offered_gnups": round(updates / span_offered / 1e9, 3) if span_offered > 0 else None}


def serving_main(args):
    cache = {}
    at_rate = serving_run(args.serving_requests, args.serving_rate, args.serving_pool, args.serving_slots,
                          args.serving_round, "serving", cache)
    saturated = serving_run(args.serving_requests, 0.0, args.serving_pool, args.serving_slots,
                            args.serving_round, "serving, saturated", cache)
    for g in cache.get("graphs", []):
        g.close()
    out = {
        "metric": "batched-serving scenarios/s + p50/p99 latency",
        "value": at_rate["batched"]["scenarios_per_s"], "unit": "scenarios/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving_mix", "requests": args.serving_requests,
                   "rate_per_s": args.serving_rate, "replicas": 16, "steps": 300, "dt": 0.1,
                   "slots": args.serving_slots, "steps_per_round": args.serving_round,
                   "parallelism": "single GPU"},
        "serving": {"at_rate": at_rate, "saturated": saturated},
    }
    print(json.dumps(out), flush=True)


MARKOV_MODEL = {"model": "sir", "beta": 0.25, "gamma": 0.15, "theta": 0.01, "p_max": 0.1, "tau_max": 1.0,
                "seed": 21}


def markov_main(args):
    import numpy as np
    import torch

    import paper_2604_22092_amd as fs
    import workloads as W

    fs.lib()
    t0 = time.perf_counter()
    rp, ci = W.erdos_renyi(1_000_000, 8.0, 1)
    n = len(rp) - 1
    seeds = W.seed_nodes(n, 100, 5)
    print(f"[markov] ER N={n} E={len(ci)} built in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    steps = args.markov_steps
    g = fs.Graph(rp, ci)
    eng = fs.Markov(g, MARKOV_MODEL, steps_per_graph=STEPS_PER_GRAPH, history_len=steps, stream=stream.cuda_stream)
    st0 = np.zeros(n, np.int32)
    st0[seeds] = 2
    eng.set_state(st0, step_index=0)
    eng.step(STEPS_PER_GRAPH)
    eng.sync()
    eng.set_state(st0, step_index=0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    eng.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    counts, taus, events = eng.history(0, steps)
    _, _, _, elapsed = eng.get_state()
    eng.close()
    g.close()
    trans = int(events.sum())
    sec = ms / 1e3
    print(f"[markov] {steps} steps ({elapsed:.1f} days): {ms:.3f} ms, {trans} transitions, "
          f"{trans / sec:.3e} transitions/s, {n * steps / sec / 1e9:.2f} GNUPS, final {counts[-1].tolist()}",
          file=sys.stderr, flush=True)
    cpu = None
    if args.cpu_budget > 0:
        import oracle
        st = st0.copy()
        done, tr, t1 = 0, 0, time.perf_counter()
        while time.perf_counter() - t1 < args.cpu_budget and done < steps:
            st, _, _, ev = oracle.markov_run((rp, ci), MARKOV_MODEL, st, 5, k0=done)
            done += 5
            tr += int(ev.sum())
        el = time.perf_counter() - t1
        cpu = {"value": tr / el, "unit": "transitions/s", "cores": 1, "kind": "oracle",
               "sample": f"steps 0..{done - 1} of the same run, single-threaded FP64 oracle, {el:.1f} s"}
    rec = {
        "metric": "Markovian engine: realized transitions per second",
        "value": round(trans / sec, 1),
        "unit": "transitions/s",
        "n_gpus": 1, "steps": steps, "warmup": STEPS_PER_GRAPH, "ms_per_step": round(ms / steps, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "er8_n1e6_sir", "graph": "Erdos-Renyi, N=1e6, mean degree 8, seed 1",
                   "model": "SIR beta=0.25 gamma=0.15", "theta": 0.01, "p_max": 0.1, "tau_max": 1.0, "seeds": 100,
                   "simulated_days": round(elapsed, 3), "transitions": trans,
                   "gnups": round(n * steps / sec / 1e9, 3), "parallelism": "single GPU"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["regular10_n1e6", "ba5_n1e6", "regular8_n1e8"],
                    default=WORKLOAD)
    ap.add_argument("--storage", choices=["fp32", "compact"], default=None,
                    help="state/age storage (default: the workload's)")
    ap.add_argument("--tune", choices=["auto", "on", "off"], default="auto",
                    help="run the autotuner (step variant and degree bins) before timing "
                         "(auto: for every workload but the default one, whose plain step is "
                         "configuration 1 as stated)")
    ap.add_argument("--tune-cache", default=None,
                    help="tune cache file: a choice cached for the run's signature is applied "
                         "without trials, a new one is appended")
    ap.add_argument("--steps", type=int, default=None,
                    help="steps per timed window (default: the workload's trajectory length); "
                         "shorter windows tile the trajectory, each timed on its own")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of the trajectory (value: their mean; CoV reported)")
    ap.add_argument("--bins", default=None,
                    help="explicit degree bins 'heavy_degree,segment_edges' (no tuning)")
    ap.add_argument("--cpu-budget", type=float, default=16.0,
                    help="seconds of oracle time for the CPU baselines, half on one core and half "
                         "on all cores (0 = skip)")
    ap.add_argument("--variant", choices=["auto", "stream", "resident", "summary"], default="auto",
                    help="step kernel variant (auto: LDS-resident bitmap when N*R <= 2^20, "
                         "else the LDS summary that screens bitmap reads)")
    ap.add_argument("--shed", choices=["none", "hazard", "density", "unit"], default="none",
                    help="shedding profile s(tau): none (s = 1), hazard (h_IR), density (log-normal), "
                         "unit (s = 1 through the shedding kernels)")
    ap.add_argument("--compaction", action="store_true", help="active-node compaction")
    ap.add_argument("--columns", choices=["auto", "plain"], default="auto",
                    help="the step's graph copy: packed columns where supported (auto) or 32-bit")
    ap.add_argument("--beta", type=float, default=None, help="override the workload's beta")
    ap.add_argument("--markov", action="store_true", help="measure the Markovian engine instead")
    ap.add_argument("--markov-steps", type=int, default=600)
    ap.add_argument("--serving", action="store_true",
                    help="measure the scenario server on the seeded request mix instead")
    ap.add_argument("--serving-requests", type=int, default=400)
    ap.add_argument("--serving-rate", type=float, default=50.0, help="Poisson arrivals per second")
    ap.add_argument("--serving-pool", type=int, default=24, help="resident pool graphs")
    ap.add_argument("--serving-slots", type=int, default=0, help="server slot limit (0 = default)")
    ap.add_argument("--serving-round", type=int, default=0, help="steps per round (0 = default)")
    ap.add_argument("--serving-sample", type=int, default=48,
                    help="requests of the short serving measurement in the default line (0 = none)")
    ap.add_argument("--serving-sample-pool", type=int, default=6,
                    help="pool graphs of the short serving measurement")
    ap.add_argument("--n", type=float, default=0,
                    help="run the workload's graph family at this many nodes instead (an N sweep)")
    ap.add_argument("--graph-cache", default=None,
                    help="directory where generated graphs are kept as .npy files and reused")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB, so a "
                         "counter profile of the same process can scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(replicas and scenarios shard across GPUs without exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving_main(args)
        return
    if args.markov:
        markov_main(args)
        return

    import numpy as np
    import torch

    import paper_2604_22092_amd as fs
    import workloads as W

    fs.lib()  # fail loudly without the HIP library
    workload = args.workload
    wl = W.WORKLOADS[workload]
    model = dict(wl["model"])
    if args.beta is not None:
        model["beta"] = args.beta
    shed = ("hazard", model["ir"], 1.0) if args.shed == "hazard" else SHEDS[args.shed]
    model["shed"] = shed
    storage = args.storage or wl["storage"]
    compact = storage == "compact"
    traj = wl["steps"]
    K = args.steps if args.steps is not None else traj
    # the captured step loop: b steps per replay (at most 50, even), so that
    # a window of K steps is replayed from the graph (K // b replays, K % b
    # single launches)
    spg = min(STEPS_PER_GRAPH, K)
    if spg > 1:
        spg -= spg % 2
    # timed windows of K steps tile the configured trajectory: a short K
    # measures the same mix of epidemic phases as the whole run
    nwin = -(-traj // K) if K < traj else 1
    t0 = time.perf_counter()
    spec = wl["graph"]
    if args.n:
        # the workload's graph family and degree at another size (an N sweep)
        spec = (spec[0], int(args.n) + (int(args.n) & 1 if spec[0] == "regular_m" else 0)) + tuple(spec[2:])
    rp, ci = load_graph(spec, args.graph_cache)
    n = len(rp) - 1
    seeds = W.seed_nodes(n, wl["seeds"], wl["seed_rng"])
    print(f"[bench] graph {workload}: N={n} E={len(ci)} built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done", file=sys.stderr,
              flush=True)
    g = fs.Graph(rp, ci)
    variant = {"auto": fs.VARIANT_AUTO, "stream": fs.VARIANT_STREAM,
               "resident": fs.VARIANT_RESIDENT, "summary": fs.VARIANT_SUMMARY}[args.variant]
    bins = tuple(int(x) for x in args.bins.split(",")) if args.bins else (0, 0)
    sim = fs.Sim.from_model(g, model, steps_per_graph=spg, stream=stream.cuda_stream,
                            variant=variant, compaction=args.compaction,
                            storage=fs.FS_STORAGE_COMPACT if compact else fs.FS_STORAGE_FP32,
                            heavy_degree=bins[0], segment_edges=bins[1],
                            history_len=max(1024, nwin * K + 1),
                            columns=fs.FS_COLUMNS_PLAIN if args.columns == "plain" else fs.FS_COLUMNS_AUTO)
    init_state = W.initial_state(n, seeds)
    init_age = np.zeros(n, np.uint16 if compact else np.float32)
    tuned = None
    if not args.bins and (args.tune == "on" or (args.tune == "auto" and workload != WORKLOAD)):
        sim.set_state(init_state, init_age, 0, step_index=0)
        sim.step(100)  # tune on a state with the epidemic under way
        sim.sync()
        tuned = sim.autotune(20, variants=args.variant == "auto", cache_path=args.tune_cache)
        print(f"[bench] autotuner: {tuned}", file=sys.stderr, flush=True)
    bins_used = sim.bins()
    variant_used = sim.variant()
    column_bits = sim.column_bits()

    # warm-up (graph instantiation, clocks), then restart the trajectory
    sim.set_state(init_state, init_age, 0, step_index=0)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()

    # each repeat runs the trajectory from the seeded start as nwin timed
    # windows of exactly K steps, each bracketed by device synchronisations
    runs = []      # per repeat: the summed window times (ms)
    win_ms = []
    wall = 0.0
    for rep in range(max(1, args.repeats)):
        sim.set_state(init_state, init_age, 0, step_index=0)
        tot = 0.0
        for w in range(nwin):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            e0.record(stream)
            sim.step(K)
            e1.record(stream)
            torch.cuda.synchronize()
            wall += time.perf_counter() - w0
            ms_w = e0.elapsed_time(e1)
            win_ms.append(ms_w)
            tot += ms_w
        runs.append(tot)
    steps_run = nwin * K
    ms = float(np.mean(runs))
    cov = float(np.std(runs) / ms) if len(runs) > 1 else 0.0
    wall /= len(runs)
    hist = sim.history(0, steps_run)
    assert np.all(hist.sum(1) == n)
    final = sim.counts(0)
    sim.close()
    g.close()

    sec = ms / 1e3
    gnups = n * steps_run / sec / 1e9
    d_mean = len(ci) / n
    b_alg = bytes_per_update(d_mean, storage)
    per_launch_s = sec / steps_run
    achieved = b_alg * n / per_launch_s / 1e9
    # the committed counters were taken in the workload's own configuration
    plain = (args.shed == "none" and not args.compaction and args.columns == "auto" and args.beta is None
             and not args.n and args.variant == "auto")
    traffic = measured_traffic(workload if storage == wl["storage"] else f"{workload}_{storage}") if plain else None
    s_frac = float(hist[:, 0].mean() / n)
    copy_gbs = copy_bandwidth(torch, dev)
    print(f"[bench] {nwin} x {K} steps (b = {spg}): {ms:.3f} ms mean of {len(runs)} (CoV {cov:.3f}, "
          f"wall {wall * 1e3:.1f} ms), {gnups:.2f} GNUPS, copy {copy_gbs:.0f} GB/s, "
          f"final counts {final.tolist()}, mean S fraction {s_frac:.3f}", file=sys.stderr, flush=True)

    cpu = None
    if args.cpu_budget > 0:
        one = cpu_baseline(rp, ci, model, seeds, args.cpu_budget / 2, compact)
        print(f"[bench] cpu baseline, one core: {one['value'] * 1e3:.1f} MNUPS", file=sys.stderr, flush=True)
        cpu = cpu_all_cores(rp, ci, model, seeds, args.cpu_budget / 2, compact)
        cpu["one_core"] = one
        print(f"[bench] cpu baseline, {cpu['cores']} cores: {cpu['value'] * 1e3:.1f} MNUPS", file=sys.stderr,
              flush=True)

    serving = None
    if args.serving_sample > 0 and workload == WORKLOAD and plain:
        cache = {}
        try:
            serving = {
                "at_rate": serving_run(args.serving_sample, args.serving_rate, args.serving_sample_pool,
                                       label="serving sample", graphs_cache=cache),
                "saturated": serving_run(args.serving_sample, 0.0, args.serving_sample_pool,
                                         label="serving sample, saturated", graphs_cache=cache),
            }
        except Exception as e:  # the step line stands on its own; the failure is reported
            serving = {"error": repr(e)}
        for gg in cache.get("graphs", []):
            gg.close()

    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_update": b_alg,
            "per_launch_us": round(per_launch_s * 1e6, 3),
            "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
            "repeats": len(runs), "cov": round(cov, 4)}
    if traffic:
        # the bytes the kernel really moves at the L2/HBM boundary (counters)
        roof["traffic_gbs"] = round(traffic / per_launch_s / 1e9, 1)
        roof["traffic_frac"] = round(traffic / per_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    rec = {
        "metric": METRIC,
        "value": round(gnups, 4),
        "unit": "GNUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms / steps_run, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",  # hazard and pressure arithmetic; compact storage changes only what is stored
        "data": "synthetic",
        "config": {"workload": workload if not args.n else f"{workload} at N={n}",
                   "graph": GRAPH_TEXT[workload] if not args.n else re.sub(r"N=[0-9e.]+", f"N={n}", GRAPH_TEXT[workload]),
                   "n": n, "edges": int(len(ci)),
                   "laws": LAW_TEXT[workload], "beta": model["beta"], "dt": model["dt"],
                   "seeds": wl["seeds"], "replicas": 1, "storage": storage,
                   "trajectory_steps": traj, "timed_windows": nwin, "window_steps": K,
                   "steps_per_graph": spg, "graph_replays_per_window": K // spg if spg else 0,
                   "eager_steps_per_window": K % spg if spg else K,
                   "kernel_variant": variant_used,
                   "column_bits": column_bits,
                   "shedding": args.shed if shed is None else [shed[0], list(shed[1]), shed[2]],
                   "compaction": args.compaction,
                   "degree_bins": list(bins_used[:2]) if bins_used[2] else None,
                   "degree_bins_from": "tuner" if tuned else ("explicit" if args.bins else "default"),
                   "autotuner": tuned,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if serving is not None:
        rec["serving"] = serving
    print(json.dumps(rec), flush=True)

if __name__ == "__main__":
    main()
