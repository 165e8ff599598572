"""CPU oracle of the GDI annealer -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The HIP library never imports, links or
calls anything here, and this package never imports the HIP library.

Contents:
  * ``gdi_oracle.c``  -- plain C implementation of the annealing schedule
    (Sec. V Alg. 3 with the deterministic readings stated in its header), built
    into ``liboracle.so`` and wrapped below with ctypes;
  * ``ref_tiny.py``   -- a second, pure-Python implementation for tiny graphs;
  * ``exhaustive.py`` -- brute-force ground states and balanced min-cuts (n <= 20).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "gdi_oracle.c")

MODE_GATED = 0
MODE_SNAPSHOT = 1
RULE_METROPOLIS = 0
RULE_PAPER = 1


def build(verbose: bool = False) -> str:
    """Compiles liboracle.so with gcc (-O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIB_PATH, SOURCE, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_int32),
        ("B", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("n_sweeps", ctypes.c_int32),
        ("start_sweep", ctypes.c_int32),
        ("replica", ctypes.c_uint32),
        ("n_threads", ctypes.c_int32),
        ("rule", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SOURCE):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P, P]
        L.oracle_philox_many.argtypes = [ctypes.c_uint64, ctypes.c_int64, P, P]
        L.oracle_threshold.argtypes = [ctypes.c_int64, ctypes.c_double]
        L.oracle_threshold.restype = ctypes.c_uint32
        L.oracle_thresholds.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_colour.argtypes = [ctypes.c_int32, P, P, P]
        L.oracle_colour.restype = ctypes.c_int32
        L.oracle_cut.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P]
        L.oracle_energy.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, ctypes.c_int64]
        L.oracle_energy.restype = ctypes.c_int64
        L.oracle_flip_delta.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32]
        L.oracle_flip_delta.restype = ctypes.c_int64
        L.oracle_anneal.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.POINTER(_Params), P, P, P, P,
                                    P, P, P, P, P, P]
        L.oracle_anneal.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def philox(seed: int, ctrs) -> np.ndarray:
    """Philox4x32-10 of each counter row (m x 4 uint32) under key = (seed lo, seed hi)."""
    c = np.ascontiguousarray(np.asarray(ctrs, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros_like(c)
    lib().oracle_philox_many(ctypes.c_uint64(seed), c.shape[0], _p(c), _p(out))
    return out


def threshold(d: int, T: float) -> int:
    return int(lib().oracle_threshold(d, T))


def thresholds(T, width: int) -> np.ndarray:
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = np.zeros((T.size, width + 1), dtype=np.uint32)
    lib().oracle_thresholds(_p(T), T.size, width, _p(out))
    return out


def colour(g) -> tuple:
    """First-fit greedy colouring in ascending id; returns (colour array, C)."""
    rp, col = _i32(g.row_ptr), _i32(g.col)
    out = np.zeros(g.n, dtype=np.int32)
    C = lib().oracle_colour(g.n, _p(rp), _p(col), _p(out))
    if C < 0:
        raise RuntimeError(f"oracle_colour failed: {C}")
    return out, C


def cut(g, spins) -> tuple:
    """(weighted cut, crossing-edge count, magnetisation) from scratch."""
    s = np.ascontiguousarray(spins, dtype=np.int8)
    cw, ce, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().oracle_cut(g.n, _p(_i32(g.row_ptr)), _p(_i32(g.col)), _p(_i32(g.w)), _p(s),
                     ctypes.byref(cw), ctypes.byref(ce), ctypes.byref(m))
    return cw.value, ce.value, m.value


def energy(g, spins, A: int, B: int) -> int:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().oracle_energy(g.n, _p(_i32(g.row_ptr)), _p(_i32(g.col)), _p(_i32(g.w)), _p(s),
                                   A, B))


def flip_delta(g, spins, A: int, B: int, i: int) -> int:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().oracle_flip_delta(g.n, _p(_i32(g.row_ptr)), _p(_i32(g.col)), _p(_i32(g.w)),
                                       _p(s), A, B, i))


def anneal(g, temps, seed: int, A: int = 1, B: int = 1, replica: int = 0, mode: int = MODE_GATED,
           start_sweep: int = 0, init=None, n_threads: int = 0, trace: bool = False,
           phase_trace: bool = False, phase_spins: bool = False, skip=None, last_flip=None,
           rule: int = RULE_METROPOLIS) -> dict:
    """Runs the oracle schedule; returns a dict with spins, M, cut, C, flips and optional traces.

    skip (n bools): nodes that make no decision in these sweeps; last_flip (int32
    array of n, updated in place): sweep of each node's last flip. With
    rule=RULE_PAPER, temps holds the flip probabilities P_f(t) of the paper's rule.
    """
    T = np.ascontiguousarray(temps, dtype=np.float64)
    S = T.size
    rp, col, w = _i32(g.row_ptr), _i32(g.col), _i32(g.w)
    prm = _Params(A=A, B=B, mode=mode, n_sweeps=S, start_sweep=start_sweep, replica=replica,
                  n_threads=n_threads, rule=rule, seed=seed)
    spins = np.zeros(g.n, dtype=np.int8)
    init_a = None if init is None else np.ascontiguousarray(init, dtype=np.int8)
    tm = np.zeros(S, dtype=np.int64) if trace else None
    tc = np.zeros(S, dtype=np.int64) if trace else None
    C = colour(g)[1]
    pm = np.zeros(S * C, dtype=np.int64) if phase_trace else None
    pc = np.zeros(S * C, dtype=np.int64) if phase_trace else None
    ps = np.zeros((S * C, g.n), dtype=np.int8) if phase_spins else None
    res = np.zeros(5, dtype=np.int64)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    if last_flip is not None and (last_flip.dtype != np.int32 or not last_flip.flags.c_contiguous):
        raise TypeError("last_flip must be a contiguous int32 array")
    rc = lib().oracle_anneal(g.n, _p(rp), _p(col), _p(w), _p(T), ctypes.byref(prm), _p(init_a),
                             _p(spins), _p(tm), _p(tc), _p(pm), _p(pc), _p(ps), _p(res), _p(sk),
                             _p(last_flip))
    if rc != 0:
        raise RuntimeError(f"oracle_anneal failed: {rc}")
    out = dict(spins=spins, M=int(res[0]), cut=int(res[1]), C=int(res[2]), flips=int(res[3]),
               sweep_s=float(res[4]) * 1e-9)
    if trace:
        out["trace_m"], out["trace_cut"] = tm, tc
    if phase_trace:
        out["phase_m"], out["phase_cut"] = pm.reshape(S, C), pc.reshape(S, C)
    if phase_spins:
        out["phase_spins"] = ps.reshape(S, C, g.n)
    return out


def max_threads() -> int:
    return int(lib().oracle_max_threads())
