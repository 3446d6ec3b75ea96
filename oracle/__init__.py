"""FP64 CPU oracle for the renewal tau-leap SEIR step (FlashSpread, arXiv 2604.22092).

TEST INFRASTRUCTURE.  This package is the reference that the HIP library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the library and its Python
binding never do.  It shares no code with the HIP path: the C sources here
(``oracle.c``, ``gillespie.c``) have their own Philox, hazards and CSR loop.

This module is argument marshalling only (ctypes over ``liboracle.so``); the
arithmetic lives in ``oracle.c`` and follows Algorithm 3, Eq. (influence),
Eq. (infectivity), Proposition 1 and the Bernoulli tau-leap rule of the paper.

Holding-time laws are given as plain tuples, the same format the workload
descriptions use:
    ("exp", rate)            constant hazard (Markovian special case)
    ("lognormal", mu, sigma) parameters of ln(tau) (Proposition 1)
    ("weibull", shape, scale)
    ("erlang", k, rate)      integer shape k

A model may name a shedding profile s(tau) of Eq. (infectivity) under the key
"shed": ("density", law, A) for s = A f(tau), ("hazard", law, A) for
s = A h(tau), with `law` one of the tuples above; absent or ("constant",)
means s == 1.

Parity: every function here is pinned by a CPU test against something other
than itself (numpy and rocRAND for Philox, scipy/mpmath for the hazards,
closed forms, brute force and an exact event-driven simulation for the step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "gillespie.c"), os.path.join(_HERE, "markov.c")]

S, E, I, R = 0, 1, 2, 3
AGE_DAYS_F32, AGE_STEPS_U16 = 0, 1
_KINDS = {"exp": 0, "lognormal": 1, "weibull": 2, "erlang": 3}


def build() -> str:
    """Compile liboracle.so with the host C compiler (always rebuilds)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
           "-o", tmp, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    """Load liboracle.so, building it first only if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class Dist(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("ei", Dist), ("ir", Dist), ("beta", ctypes.c_double),
                ("dt", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("age_mode", ctypes.c_int32), ("shed_mode", ctypes.c_int32),
                ("shed", Dist), ("shed_scale", ctypes.c_double)]


SHED_MODES = {"constant": 0, "density": 1, "hazard": 2}


def make_dist(spec) -> Dist:
    kind = spec[0]
    if kind == "exp":
        return Dist(_KINDS[kind], 0, float(spec[1]), 0.0)
    if kind == "lognormal":
        return Dist(_KINDS[kind], 0, float(spec[1]), float(spec[2]))
    if kind == "weibull":
        return Dist(_KINDS[kind], 0, float(spec[1]), float(spec[2]))
    if kind == "erlang":
        return Dist(_KINDS[kind], int(spec[1]), float(spec[2]), 0.0)
    raise ValueError(f"unknown holding-time law {spec!r}")


def make_params(model: dict, age_mode: int = AGE_DAYS_F32) -> Params:
    shed = model.get("shed") or ("constant",)
    mode = SHED_MODES[shed[0]]
    law = make_dist(shed[1]) if mode else Dist(0, 0, 0.0, 0.0)
    scale = float(shed[2]) if mode else 1.0
    return Params(make_dist(model["ei"]), make_dist(model["ir"]), float(model["beta"]),
                  float(model["dt"]), int(model.get("seed", 0)) & (2**64 - 1), int(age_mode),
                  mode, law, scale)


class MarkovParams(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("pad", ctypes.c_int32), ("beta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("gamma", ctypes.c_double), ("theta", ctypes.c_double),
                ("p_max", ctypes.c_double), ("tau_max", ctypes.c_double), ("seed", ctypes.c_uint64)]


MARKOV_MODELS = {"seir": 0, "sir": 1, "sis": 2}


def make_markov_params(m: dict) -> MarkovParams:
    """m: {"model": "seir"|"sir"|"sis", "beta", "sigma" (SEIR), "gamma",
    "theta", "p_max", "tau_max", "seed"}."""
    return MarkovParams(MARKOV_MODELS[m["model"]], 0, float(m["beta"]), float(m.get("sigma", 0.0)),
                        float(m["gamma"]), float(m["theta"]), float(m["p_max"]), float(m["tau_max"]),
                        int(m.get("seed", 0)) & (2**64 - 1))


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32


def _declare(L):
    L.or_philox4x32_10_many.argtypes = [_I64, _P, _P, _P]
    L.or_philox4x64_10_many.argtypes = [_I64, _P, _P, _P]
    L.or_uniform.argtypes = [_U64, _I64, _U64, _U32]
    L.or_uniform.restype = ctypes.c_double
    L.or_erfcx_many.argtypes = [_I64, _P, _P]
    L.or_hazard_many.argtypes = [ctypes.POINTER(Dist), _I64, _P, _P]
    L.or_density_many.argtypes = [ctypes.POINTER(Dist), _I64, _P, _P]
    L.or_infectivity.argtypes = [_I64, ctypes.POINTER(Params), _P, _P, _P, _P]
    L.or_binary16_many.argtypes = [_I64, _P, _P]
    L.or_step.argtypes = [_I64, _P, _P, _P, ctypes.POINTER(Params), _U64, _U32, _P, _P, _P,
                          _P, _P, _P, _P, _P, _P]
    L.or_step_nodes.argtypes = [_I64, _P, _P, _P, ctypes.POINTER(Params), _U64, _U32, _P, _P,
                                _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P]
    L.or_run.argtypes = [_I64, _P, _P, _P, ctypes.POINTER(Params), _U64, _I64, _U32, _P, _P,
                         _P, _P, _P]
    L.or_next_dt.argtypes = [ctypes.c_double] * 4
    L.or_next_dt.restype = ctypes.c_double
    L.or_run_adaptive.argtypes = [_I64, _P, _P, _P, ctypes.POINTER(Params), ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _U64, _I64, _U32, _P, _P, _P,
                                  _P, _P]
    L.mk_influence.argtypes = [_I64, _P, _P, _P, _P]
    L.mk_tau.argtypes = [ctypes.POINTER(MarkovParams), _I64, _P, _P, _P, _P]
    L.mk_tau.restype = ctypes.c_double
    L.mk_step.argtypes = [_I64, _P, _P, ctypes.POINTER(MarkovParams), _U64, _P, _P, _P, _P, _P, _P, _P]
    L.mk_step.restype = ctypes.c_double
    L.mk_run.argtypes = [_I64, _P, _P, ctypes.POINTER(MarkovParams), _U64, _I64, _P, _P, _P, _P, _P]
    L.gx_run.argtypes = [_I64, _P, _P, _P, ctypes.POINTER(Dist), ctypes.POINTER(Dist),
                         ctypes.c_double, ctypes.c_double, _P, _U64, _P, _P, _I64, _P, _P]
    L.gx_run.restype = _I64
    L.gx_run_many.argtypes = [_I64, _I64, _P, _P, _P, ctypes.POINTER(Dist),
                              ctypes.POINTER(Dist), ctypes.c_double, ctypes.c_double, _P,
                              _U64, _P, _P]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------- RNG

def philox4x32(ctr, key) -> np.ndarray:
    """Philox4x32-10 of each row of ctr (n x 4 uint32) under key (2 uint32)."""
    ctr = _c(np.atleast_2d(ctr), np.uint32)
    key = _c(key, np.uint32)
    out = np.empty_like(ctr)
    lib().or_philox4x32_10_many(len(ctr), _ptr(ctr), _ptr(key), _ptr(out))
    return out


def philox4x64(ctr, key) -> np.ndarray:
    """Philox4x64-10 of each row of ctr (n x 4 uint64) under key (2 uint64)."""
    ctr = _c(np.atleast_2d(ctr), np.uint64)
    key = _c(key, np.uint64)
    out = np.empty_like(ctr)
    lib().or_philox4x64_10_many(len(ctr), _ptr(ctr), _ptr(key), _ptr(out))
    return out


def uniforms(seed: int, nodes, step: int, replica: int) -> np.ndarray:
    """The per-node uniforms u of one step (word 0 of Philox, top 24 bits)."""
    nodes = np.asarray(nodes, dtype=np.int64)
    ctr = np.zeros((len(nodes), 4), dtype=np.uint32)
    ctr[:, 0] = nodes.astype(np.uint32)
    ctr[:, 1] = np.uint32(step & 0xFFFFFFFF)
    ctr[:, 2] = np.uint32(replica)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    w = philox4x32(ctr, key)[:, 0]
    return (w >> np.uint32(8)).astype(np.float64) * 2.0**-24


# ----------------------------------------------------------------------- hazards

def erfcx(z) -> np.ndarray:
    z = _c(np.atleast_1d(z), np.float64)
    out = np.empty_like(z)
    lib().or_erfcx_many(len(z), _ptr(z), _ptr(out))
    return out


def hazard(spec, tau) -> np.ndarray:
    tau = _c(np.atleast_1d(tau), np.float64)
    out = np.empty_like(tau)
    d = make_dist(spec)
    lib().or_hazard_many(ctypes.byref(d), len(tau), _ptr(tau), _ptr(out))
    return out


def density(spec, tau) -> np.ndarray:
    """Density f(tau) of a holding-time law (shedding profiles s = A f)."""
    tau = _c(np.atleast_1d(tau), np.float64)
    out = np.empty_like(tau)
    d = make_dist(spec)
    lib().or_density_many(ctypes.byref(d), len(tau), _ptr(tau), _ptr(out))
    return out


def binary16(x) -> np.ndarray:
    """x rounded to the nearest IEEE binary16 value (ties to even), as float64."""
    a = _c(x, np.float64)
    out = np.empty_like(a)
    lib().or_binary16_many(len(a), _ptr(a), _ptr(out))
    return out


def infectivity(model: dict, state, age, compact: bool = False) -> np.ndarray:
    """iota_i = s(tau_i) 1{X_i = I} of Eq. (infectivity), from a state and age
    (stored in binary16 under compact storage)."""
    st = _c(state, np.int32)
    n = len(st)
    p = make_params(model, AGE_STEPS_U16 if compact else AGE_DAYS_F32)
    ad = None if compact else _c(age, np.float32)
    ag = _c(age, np.uint16) if compact else None
    out = np.empty(n, dtype=np.float64)
    lib().or_infectivity(n, ctypes.byref(p), _ptr(st), _ptr(ad), _ptr(ag), _ptr(out))
    return out


# -------------------------------------------------------------------------- step

def _graph(graph):
    row_ptr, col_ind = graph[0], graph[1]
    weights = graph[2] if len(graph) > 2 else None
    return _c(row_ptr, np.int32), _c(col_ind, np.int32), _c(weights, np.float32)


def step(graph, model: dict, state, age, iota, step_index: int, replica: int = 0,
         compact: bool = False) -> dict:
    """One step from (state, age, iota); returns the new arrays plus logs.

    age is float32 days (compact=False) or uint16 step counts (compact=True).
    iota is the start-of-step infectivity s(tau) 1{X = I} (see infectivity()).
    """
    rp, ci, w = _graph(graph)
    n = len(rp) - 1
    st = np.array(state, dtype=np.int32, copy=True)
    p = make_params(model, AGE_STEPS_U16 if compact else AGE_DAYS_F32)
    ad = None if compact else np.array(age, dtype=np.float32, copy=True)
    ag = np.array(age, dtype=np.uint16, copy=True) if compact else None
    io = _c(iota, np.float64)
    io_out = np.empty(n, dtype=np.float64)
    counts = np.zeros(4, dtype=np.int64)
    lam = np.empty(n, dtype=np.float64)
    q = np.empty(n, dtype=np.float64)
    u = np.empty(n, dtype=np.float64)
    lib().or_step(n, _ptr(rp), _ptr(ci), _ptr(w), ctypes.byref(p), int(step_index) & (2**64 - 1),
                  int(replica), _ptr(st), _ptr(ad), _ptr(ag), _ptr(io), _ptr(io_out),
                  _ptr(counts), _ptr(lam), _ptr(q), _ptr(u))
    return {"state": st, "age": ag if compact else ad, "iota": io_out, "counts": counts,
            "lam": lam, "q": q, "u": u}


def step_nodes(graph, model: dict, state, age, iota, step_index: int, nodes,
               replica: int = 0, compact: bool = False) -> dict:
    """The step's outcome for the listed nodes only, from a full snapshot."""
    rp, ci, w = _graph(graph)
    n = len(rp) - 1
    nodes = _c(nodes, np.int64)
    m = len(nodes)
    st = _c(state, np.int32)
    p = make_params(model, AGE_STEPS_U16 if compact else AGE_DAYS_F32)
    ad = None if compact else _c(age, np.float32)
    ag = _c(age, np.uint16) if compact else None
    io = _c(iota, np.float64)
    out_state = np.empty(m, dtype=np.int32)
    out_ad = None if compact else np.empty(m, dtype=np.float32)
    out_ag = np.empty(m, dtype=np.uint16) if compact else None
    lam = np.empty(m, dtype=np.float64)
    q = np.empty(m, dtype=np.float64)
    u = np.empty(m, dtype=np.float64)
    lib().or_step_nodes(n, _ptr(rp), _ptr(ci), _ptr(w), ctypes.byref(p),
                        int(step_index) & (2**64 - 1), int(replica), _ptr(st), _ptr(ad),
                        _ptr(ag), _ptr(io), m, _ptr(nodes), _ptr(out_state), _ptr(out_ad),
                        _ptr(out_ag), _ptr(lam), _ptr(q), _ptr(u))
    return {"state": out_state, "age": out_ag if compact else out_ad, "lam": lam, "q": q,
            "u": u}


def run(graph, model: dict, state, age, n_steps: int, step0: int = 0, replica: int = 0,
        compact: bool = False):
    """A trajectory of n_steps steps; returns (state, age, history[n_steps, 4])."""
    rp, ci, w = _graph(graph)
    n = len(rp) - 1
    st = np.array(state, dtype=np.int32, copy=True)
    p = make_params(model, AGE_STEPS_U16 if compact else AGE_DAYS_F32)
    ad = None if compact else np.array(age, dtype=np.float32, copy=True)
    ag = np.array(age, dtype=np.uint16, copy=True) if compact else None
    scratch = np.empty(2 * n, dtype=np.float64)
    hist = np.zeros((n_steps, 4), dtype=np.int64)
    lib().or_run(n, _ptr(rp), _ptr(ci), _ptr(w), ctypes.byref(p), int(step0), int(n_steps),
                 int(replica), _ptr(st), _ptr(ad), _ptr(ag), _ptr(scratch), _ptr(hist))
    return st, (ag if compact else ad), hist


def next_dt(lam_max: float, eps: float, dt_max: float, delta: float = 0.0) -> float:
    """The adaptive step after a step whose largest rate was lam_max."""
    return lib().or_next_dt(float(lam_max), float(eps), float(dt_max), float(delta))


def run_adaptive(graph, model: dict, state, age, n_steps: int, eps: float, dt_max: float,
                 delta: float = 0.0, step0: int = 0, replica: int = 0):
    """An adaptive-step trajectory (ages in days; model["dt"] is ignored):
    returns (state, age, history[n_steps, 4], dts[n_steps])."""
    rp, ci, w = _graph(graph)
    n = len(rp) - 1
    st = np.array(state, dtype=np.int32, copy=True)
    p = make_params(dict(model, dt=dt_max), AGE_DAYS_F32)
    ad = np.array(age, dtype=np.float32, copy=True)
    scratch = np.empty(3 * n, dtype=np.float64)
    hist = np.zeros((n_steps, 4), dtype=np.int64)
    dts = np.zeros(n_steps, dtype=np.float64)
    lib().or_run_adaptive(n, _ptr(rp), _ptr(ci), _ptr(w), ctypes.byref(p), float(eps), float(dt_max),
                          float(delta), int(step0), int(n_steps), int(replica), _ptr(st), _ptr(ad),
                          _ptr(scratch), _ptr(hist), _ptr(dts))
    return st, ad, hist, dts


# ----------------------------------------------------------- exact simulation

def gillespie(graph, ei, ir, beta: float, t_end: float, init_state, seed: int,
              reps: int):
    """Exact event-driven realisations; returns (peak_I[reps], counts[reps, 4])."""
    rp, ci, w = _graph(graph)
    n = len(rp) - 1
    st = _c(init_state, np.int32)
    dei, dir_ = make_dist(ei), make_dist(ir)
    peaks = np.zeros(reps, dtype=np.int64)
    counts = np.zeros((reps, 4), dtype=np.int64)
    lib().gx_run_many(int(reps), n, _ptr(rp), _ptr(ci), _ptr(w), ctypes.byref(dei),
                      ctypes.byref(dir_), float(beta), float(t_end), _ptr(st), int(seed),
                      _ptr(peaks), _ptr(counts))
    return peaks, counts


# ------------------------------------------------------------ Markovian engine

def markov_influence(graph, state) -> np.ndarray:
    """Infectious in-neighbours of every node (unit weights)."""
    rp, ci, _ = _graph(graph)
    st = _c(state, np.int32)
    out = np.empty(len(rp) - 1, dtype=np.int32)
    lib().mk_influence(len(rp) - 1, _ptr(rp), _ptr(ci), _ptr(st), _ptr(out))
    return out


def markov_tau(graph, m: dict, state):
    """(tau, Lambda, max lambda) of the step from `state`."""
    rp, ci, _ = _graph(graph)
    st = _c(state, np.int32)
    infl = markov_influence(graph, st)
    L = ctypes.c_double()
    M = ctypes.c_double()
    p = make_markov_params(m)
    tau = lib().mk_tau(ctypes.byref(p), len(st), _ptr(st), _ptr(infl), ctypes.byref(L), ctypes.byref(M))
    return tau, L.value, M.value


def markov_step(graph, m: dict, state, k: int) -> dict:
    """One step k of the Markovian engine from `state`."""
    rp, ci, _ = _graph(graph)
    n = len(rp) - 1
    st = np.array(state, dtype=np.int32, copy=True)
    infl = markov_influence(graph, st)
    counts = np.zeros(4, np.int64)
    ev = ctypes.c_int64()
    lam = np.empty(n)
    q = np.empty(n)
    u = np.empty(n)
    p = make_markov_params(m)
    tau = lib().mk_step(n, _ptr(rp), _ptr(ci), ctypes.byref(p), int(k), _ptr(st), _ptr(infl), _ptr(counts),
                        ctypes.byref(ev), _ptr(lam), _ptr(q), _ptr(u))
    return {"state": st, "infl": infl, "counts": counts, "events": ev.value, "tau": tau, "lam": lam, "p": q,
            "u": u}


def markov_run(graph, m: dict, state, n_steps: int, k0: int = 0):
    """n_steps steps; returns (state, history[n_steps, 4], taus[n_steps], events[n_steps])."""
    rp, ci, _ = _graph(graph)
    n = len(rp) - 1
    st = np.array(state, dtype=np.int32, copy=True)
    scratch = np.empty(n, np.int32)
    hist = np.zeros((n_steps, 4), np.int64)
    taus = np.zeros(n_steps)
    evs = np.zeros(n_steps, np.int64)
    p = make_markov_params(m)
    lib().mk_run(n, _ptr(rp), _ptr(ci), ctypes.byref(p), int(k0), int(n_steps), _ptr(st), _ptr(scratch),
                 _ptr(hist), _ptr(taus), _ptr(evs))
    return st, hist, taus, evs
