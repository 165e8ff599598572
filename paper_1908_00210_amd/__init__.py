"""Python binding of libgdi.so, the MI355X GDI annealer (C ABI in include/gdi.h).

Argument marshalling only: every step of the annealing path runs in the HIP
kernels of libgdi.so. There is no CPU fallback: if the library is missing or no
gfx950 device is present, the calls raise.

Host-array entry points take numpy arrays; the ``*_dev`` entry points take
device pointers (e.g. ``torch.Tensor.data_ptr()`` of a tensor on ``cuda:0``) and
run on the stream given to :func:`set_stream`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "GdiError", "lib", "LIB_PATH", "BAL_GATED", "BAL_SNAPSHOT", "ACCEPT_METROPOLIS", "ACCEPT_PAPER", "FLAG_DENSE_BALANCE", "FLAG_RACY", "SCOPE_AUTO", "SCOPE_WORKGROUP",
    "SCOPE_GRID", "SCOPE_GRID_FENCED", "Schedule", "Tuning", "Result", "GraphInfo", "create", "destroy", "anneal",
    "anneal_dev", "cut", "cut_dev", "last_result", "set_stream", "set_tuning", "get_info",
    "get_colouring", "colour_csr", "threshold_table", "philox4x32_10", "version", "Annealer",
    "Instance", "anneal_batch", "autotune_batch", "MLP_PARAMS", "SKIP_NONE", "SKIP_MLP", "SKIP_HEURISTIC",
    "LearnedCfg", "LearnedResult", "TrainCfg", "anneal_learned", "collect_traces", "mlp_init", "mlp_train",
    "mlp_forward", "mlp_gradient", "mlp_unflatten",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgdi.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, ESTATE, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
_NAMES = {EINVAL: "GDI_EINVAL", ERANGE: "GDI_ERANGE", ENOMEM: "GDI_ENOMEM", EDEVICE: "GDI_EDEVICE",
          ESTATE: "GDI_ESTATE", ETIMEOUT: "GDI_ETIMEOUT"}
BAL_GATED, BAL_SNAPSHOT = 0, 1
ACCEPT_METROPOLIS, ACCEPT_PAPER = 0, 1
FLAG_DENSE_BALANCE = 1
FLAG_RACY = 2
SCOPE_AUTO, SCOPE_WORKGROUP, SCOPE_GRID, SCOPE_GRID_FENCED = 0, 1, 2, 3


class GdiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Schedule(ctypes.Structure):
    _fields_ = [
        ("n_sweeps", ctypes.c_uint32),
        ("start_sweep", ctypes.c_uint32),
        ("temps", ctypes.c_void_p),
        ("A", ctypes.c_int32),
        ("B", ctypes.c_int32),
        ("replica", ctypes.c_uint32),
        ("balance_mode", ctypes.c_uint32),
        ("init_spins", ctypes.c_void_p),
        ("trace_m", ctypes.c_void_p),
        ("trace_cut", ctypes.c_void_p),
        ("acceptance", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("scope", ctypes.c_uint32), ("block", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("lanes_per_node", ctypes.c_uint32), ("tail_max", ctypes.c_int32), ("spin_limit", ctypes.c_uint64),
                ("leaders", ctypes.c_int32), ("general_weights", ctypes.c_int32), ("csr_lds", ctypes.c_int32),
                ("batch_members", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [
        ("magnetization", ctypes.c_int64),
        ("cut_weighted", ctypes.c_int64),
        ("sweep_ms", ctypes.c_double),
        ("n_colours", ctypes.c_uint32),
        ("scope", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("lanes_per_node", ctypes.c_uint32),
        ("table_width", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("replica", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("spins_out", ctypes.c_void_p), ("magnetization", ctypes.c_int64),
                ("cut_weighted", ctypes.c_int64)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_colours", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("max_abs_wdeg", ctypes.c_int64), ("max_degree", ctypes.c_int32), ("pad", ctypes.c_int32)]


# network weights travel as one flat float32 array in gdi_mlp_weights order:
# w1[64][6], b1[64], w2[64][64], b2[64], w3[64], b3
MLP_PARAMS = 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1
SKIP_NONE, SKIP_MLP, SKIP_HEURISTIC = 0, 1, 2


class LearnedCfg(ctypes.Structure):
    _fields_ = [("k_full", ctypes.c_uint32), ("skip_mode", ctypes.c_uint32), ("skip_threshold", ctypes.c_float),
                ("heuristic_k", ctypes.c_uint32), ("mask_trace", ctypes.c_void_p), ("active_max", ctypes.c_int32),
                ("learn_from", ctypes.c_uint32)]


class LearnedResult(ctypes.Structure):
    _fields_ = [("magnetization", ctypes.c_int64), ("cut_weighted", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("node_visits", ctypes.c_uint64), ("node_skips", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


# every symbol include/gdi.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
SIGNATURES = {
    "gdi_create": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "gdi_destroy": (None, [_P]),
    "gdi_set_stream": (ctypes.c_int, [_P, _P]),
    "gdi_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(Tuning)]),
    "gdi_anneal": (ctypes.c_int, [_P, ctypes.POINTER(Schedule), ctypes.c_uint64, _P]),
    "gdi_anneal_dev": (ctypes.c_int, [_P, ctypes.POINTER(Schedule), ctypes.c_uint64, _P]),
    "gdi_last_result": (ctypes.c_int, [_P, ctypes.POINTER(Result)]),
    "gdi_cut": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "gdi_cut_dev": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "gdi_cut_dev_noalloc": (ctypes.c_int, [_P, _P, _P]),
    "gdi_get_info": (ctypes.c_int, [_P, ctypes.POINTER(GraphInfo)]),
    "gdi_get_colouring": (ctypes.c_int, [_P, _P, _P]),
    "gdi_colour_csr": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    "gdi_threshold_table": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_int32, _P]),
    "gdi_philox4x32_10": (ctypes.c_int, [ctypes.c_uint64, _P, _P]),
    "gdi_anneal_batch": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_uint32, ctypes.POINTER(Schedule),
                                        ctypes.c_uint64, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)]),
    "gdi_anneal_batch_dev": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_uint32, ctypes.POINTER(Schedule),
                                            ctypes.c_uint64, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)]),
    "gdi_autotune_batch": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_uint32, ctypes.POINTER(Schedule),
                                          ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(Tuning),
                                          ctypes.POINTER(ctypes.c_double)]),
    "gdi_autotune": (ctypes.c_int, [_P, ctypes.POINTER(Schedule), ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                    ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)]),
    "gdi_tune_cache_load": (ctypes.c_int, [ctypes.c_char_p]),
    "gdi_tune_cache_save": (ctypes.c_int, [ctypes.c_char_p]),
    "gdi_tune_cache_clear": (ctypes.c_int, []),
    "gdi_tune_cache_size": (ctypes.c_int, []),
    "gdi_anneal_learned": (ctypes.c_int, [_P, ctypes.POINTER(Schedule), ctypes.c_uint64, _P,
                                          ctypes.POINTER(LearnedCfg), _P, ctypes.POINTER(LearnedResult)]),
    "gdi_collect_traces": (ctypes.c_int, [_P, ctypes.POINTER(Schedule), ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "gdi_mlp_init": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "gdi_mlp_train": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.POINTER(TrainCfg), _P, _P]),
    "gdi_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_uint32, _P, _P]),
    "gdi_mlp_gradient": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, _P, ctypes.POINTER(ctypes.c_float), _P]),
    "gdi_last_error": (ctypes.c_char_p, []),
    "gdi_version": (ctypes.c_int, []),
}

_lib = None


def lib():
    """Loads libgdi.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1908_00210_amd/build.py "
                              "or __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise GdiError(rc, lib().gdi_last_error().decode(errors="replace"))
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def version() -> int:
    return lib().gdi_version()


def create(row_ptr, col, w, n: int):
    """gdi_create on a symmetric int32 CSR; returns the opaque handle (an int)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().gdi_create(_ptr(rp), _ptr(ci), _ptr(ww), int(n), ctypes.byref(h)))
    return h.value


def destroy(h):
    lib().gdi_destroy(h)


def set_stream(h, stream_ptr: int | None):
    _check(lib().gdi_set_stream(h, stream_ptr))


def set_tuning(h, scope: int = 0, block: int = 0, grid: int = 0, lanes_per_node: int = 0,
               spin_limit: int = 0, tail_max: int = 0, leaders: int = 0, general_weights: int = 0, csr_lds: int = 0,
               reset=False):
    if reset:
        _check(lib().gdi_set_tuning(h, None))
        return
    t = Tuning(scope, block, grid, lanes_per_node, tail_max, spin_limit, leaders, general_weights, csr_lds)
    _check(lib().gdi_set_tuning(h, ctypes.byref(t)))


def _schedule(temps, A, B, replica, mode, start_sweep, init, trace_m, trace_cut, acceptance=ACCEPT_METROPOLIS,
              flags=0):
    T = np.ascontiguousarray(temps, dtype=np.float64)
    s = Schedule(n_sweeps=T.size, start_sweep=start_sweep, temps=T.ctypes.data, A=A, B=B,
                 replica=replica, balance_mode=mode,
                 init_spins=None if init is None else init.ctypes.data,
                 trace_m=None if trace_m is None else trace_m.ctypes.data,
                 trace_cut=None if trace_cut is None else trace_cut.ctypes.data,
                 acceptance=acceptance, flags=flags)
    return s, T


def anneal(h, n: int, temps, seed: int, A: int = 1, B: int = 1, replica: int = 0, mode: int = BAL_GATED,
           start_sweep: int = 0, init=None, trace: bool = False, acceptance: int = ACCEPT_METROPOLIS,
           flags: int = 0) -> dict:
    """gdi_anneal: returns dict(spins (original order), M, cut, result, [trace_m, trace_cut]).

    temps: temperatures (Metropolis) or flip probabilities P_f(t) (acceptance=ACCEPT_PAPER)."""
    T = np.ascontiguousarray(temps, dtype=np.float64)
    init_a = None if init is None else np.ascontiguousarray(init, dtype=np.int8)
    tm = np.zeros(T.size, dtype=np.int64) if trace else None
    tc = np.zeros(T.size, dtype=np.int64) if trace else None
    s, T = _schedule(T, A, B, replica, mode, start_sweep, init_a, tm, tc, acceptance, flags)
    out = np.zeros(n, dtype=np.int8)
    _check(lib().gdi_anneal(h, ctypes.byref(s), ctypes.c_uint64(seed), _ptr(out)))
    r = last_result(h)
    d = dict(spins=out, M=r.magnetization, cut=r.cut_weighted, result=r.as_dict())
    if trace:
        d["trace_m"], d["trace_cut"] = tm, tc
    return d


def anneal_dev(h, temps, seed: int, d_spins_out: int, A: int = 1, B: int = 1, replica: int = 0,
               mode: int = BAL_GATED, start_sweep: int = 0, init=None, acceptance: int = ACCEPT_METROPOLIS,
               flags: int = 0):
    """gdi_anneal_dev: enqueues the anneal on the handle's stream; d_spins_out is a device pointer."""
    init_a = None if init is None else np.ascontiguousarray(init, dtype=np.int8)
    s, T = _schedule(temps, A, B, replica, mode, start_sweep, init_a, None, None, acceptance, flags)
    _check(lib().gdi_anneal_dev(h, ctypes.byref(s), ctypes.c_uint64(seed), ctypes.c_void_p(d_spins_out)))


def last_result(h) -> Result:
    r = Result()
    _check(lib().gdi_last_result(h, ctypes.byref(r)))
    return r


def cut(h, spins) -> tuple:
    """(weighted cut, crossing edges, M) of host spins (original order)."""
    s = np.ascontiguousarray(spins, dtype=np.int8)
    cw, ce, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().gdi_cut(h, _ptr(s), ctypes.byref(cw), ctypes.byref(ce), ctypes.byref(m)))
    return cw.value, ce.value, m.value


def cut_dev(h, d_spins: int) -> tuple:
    cw, ce, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().gdi_cut_dev(h, ctypes.c_void_p(d_spins), ctypes.byref(cw), ctypes.byref(ce), ctypes.byref(m)))
    return cw.value, ce.value, m.value


def cut_dev_noalloc(h, d_spins: int, d_out: int) -> None:
    """gdi_cut_dev_noalloc: writes (weighted cut, crossing count, M) as 3 int64 to d_out (device)."""
    _check(lib().gdi_cut_dev_noalloc(h, ctypes.c_void_p(d_spins), ctypes.c_void_p(d_out)))


def get_info(h) -> GraphInfo:
    i = GraphInfo()
    _check(lib().gdi_get_info(h, ctypes.byref(i)))
    return i


def get_colouring(h, n: int, n_colours: int) -> tuple:
    col = np.zeros(n, dtype=np.int32)
    sizes = np.zeros(n_colours, dtype=np.int32)
    _check(lib().gdi_get_colouring(h, _ptr(col), _ptr(sizes)))
    return col, sizes


def colour_csr(row_ptr, col, n: int) -> tuple:
    """Host-only first-fit colouring: (colour array, number of colours)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    out = np.zeros(n, dtype=np.int32)
    C = _check(lib().gdi_colour_csr(_ptr(rp), _ptr(ci), int(n), _ptr(out)))
    return out, C


def threshold_table(temps, width: int) -> np.ndarray:
    T = np.ascontiguousarray(temps, dtype=np.float64)
    out = np.zeros((T.size, width + 1), dtype=np.uint32)
    _check(lib().gdi_threshold_table(_ptr(T), T.size, int(width), _ptr(out)))
    return out


def philox4x32_10(seed: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _check(lib().gdi_philox4x32_10(ctypes.c_uint64(seed), _ptr(c), _ptr(out)))
    return out


def anneal_batch(items, temps, seed: int, A: int = 1, B: int = 1, mode: int = BAL_GATED, tune: dict | None = None,
                 outputs: bool = True, device_outputs=None, acceptance: int = ACCEPT_METROPOLIS) -> dict:
    """gdi_anneal_batch over items = [(handle, n, replica), ...].

    Returns dict(spins=[arrays or None], M=[...], cut=[...], kernel_ms). With
    device_outputs (a list of device pointers) the spins land there instead.
    """
    k = len(items)
    arr = (Instance * k)()
    outs = []
    for i, (h, n, rep) in enumerate(items):
        arr[i].graph = h
        arr[i].replica = rep
        if device_outputs is not None:
            arr[i].spins_out = device_outputs[i]
            outs.append(None)
        elif outputs:
            o = np.zeros(n, dtype=np.int8)
            outs.append(o)
            arr[i].spins_out = o.ctypes.data
        else:
            outs.append(None)
            arr[i].spins_out = None
    s, T = _schedule(temps, A, B, 0, mode, 0, None, None, None, acceptance)
    t = None if tune is None else ctypes.byref(Tuning(tune.get("scope", 0), tune.get("block", 0), tune.get("grid", 0),
                                                       tune.get("lanes_per_node", 0), 0, 0, 0, 0, 0,
                                                       tune.get("batch_members", 0)))
    ms = ctypes.c_double()
    fn = lib().gdi_anneal_batch_dev if device_outputs is not None else lib().gdi_anneal_batch
    _check(fn(arr, k, ctypes.byref(s), ctypes.c_uint64(seed), t, ctypes.byref(ms)))
    return dict(spins=outs, M=[arr[i].magnetization for i in range(k)], cut=[arr[i].cut_weighted for i in range(k)],
                kernel_ms=ms.value)


def autotune_batch(items, temps, seed: int, probe_sweeps: int, A: int = 1, B: int = 1, mode: int = BAL_GATED) -> tuple:
    """gdi_autotune_batch: returns (tuning dict, probe ms)."""
    k = len(items)
    arr = (Instance * k)()
    for i, (h, n, rep) in enumerate(items):
        arr[i].graph = h
        arr[i].replica = rep
    s, T = _schedule(temps, A, B, 0, mode, 0, None, None, None)
    best = Tuning()
    ms = ctypes.c_double()
    _check(lib().gdi_autotune_batch(arr, k, ctypes.byref(s), ctypes.c_uint64(seed), probe_sweeps, ctypes.byref(best),
                                    ctypes.byref(ms)))
    return _tuning_dict(best), ms.value


def _tuning_dict(t: Tuning) -> dict:
    """The non-default fields of a Tuning (the keys set_tuning and anneal_batch take)."""
    keys = ("scope", "block", "grid", "lanes_per_node", "tail_max", "leaders", "general_weights", "csr_lds",
            "batch_members")
    return {k: int(getattr(t, k)) for k in keys if getattr(t, k)}


def autotune(h, temps, seed: int, probe_sweeps: int = 0, use_cache: bool = False, A: int = 1, B: int = 1,
             mode: int = BAL_GATED) -> tuple:
    """gdi_autotune: installs the fastest launch choice on the handle; returns (tuning dict, probe ms)."""
    s, T = _schedule(temps, A, B, 0, mode, 0, None, None, None)
    best = Tuning()
    ms = ctypes.c_double()
    _check(lib().gdi_autotune(h, ctypes.byref(s), ctypes.c_uint64(seed), int(probe_sweeps), int(bool(use_cache)),
                              ctypes.byref(best), ctypes.byref(ms)))
    return _tuning_dict(best), ms.value


def tune_cache_load(path: str):
    _check(lib().gdi_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path: str):
    _check(lib().gdi_tune_cache_save(os.fsencode(path)))


def tune_cache_clear():
    _check(lib().gdi_tune_cache_clear())


def tune_cache_size() -> int:
    return _check(lib().gdi_tune_cache_size())


def _weights(w) -> np.ndarray:
    a = np.ascontiguousarray(w, dtype=np.float32)
    if a.size != MLP_PARAMS:
        raise ValueError(f"network weights must hold {MLP_PARAMS} floats")
    return a


def mlp_unflatten(w) -> dict:
    """Views of a flat weight array as w1 (64x6), b1, w2 (64x64), b2, w3, b3."""
    w = np.asarray(w)
    o, d = 0, {}
    for name, shape in (("w1", (64, 6)), ("b1", (64,)), ("w2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", ())):
        k = int(np.prod(shape)) if shape else 1
        d[name] = w[o:o + k].reshape(shape) if shape else w[o]
        o += k
    return d


def mlp_init(seed: int) -> np.ndarray:
    w = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(lib().gdi_mlp_init(_ptr(w), ctypes.c_uint64(seed)))
    return w


def anneal_learned(h, n: int, temps, seed: int, k_full: int, skip_mode: int = SKIP_NONE, weights=None,
                   skip_threshold: float = 0.5, heuristic_k: int = 1, A: int = 1, B: int = 1, replica: int = 0,
                   mode: int = BAL_GATED, start_sweep: int = 0, init=None, mask_trace: bool = False,
                   active_max: int = 0, learn_from: int = 0) -> dict:
    """gdi_anneal_learned: dict(spins, M, cut, result, [masks (blocks x n uint8)]).

    active_max: 0 = automatic, < 0 = never use the one-workgroup active-set sweep,
    > 0 = use it for masked sweeps with at most that many active nodes."""
    T = np.ascontiguousarray(temps, dtype=np.float64)
    init_a = None if init is None else np.ascontiguousarray(init, dtype=np.int8)
    s, T = _schedule(T, A, B, replica, mode, start_sweep, init_a, None, None)
    w = None if weights is None else _weights(weights)
    b0 = min(T.size, max(start_sweep, learn_from))
    rows = (T.size - b0 + k_full - 1) // k_full if k_full > 0 else 0
    masks = np.zeros((rows, n), dtype=np.uint8) if mask_trace else None
    cfg = LearnedCfg(k_full, skip_mode, skip_threshold, heuristic_k, None if masks is None else masks.ctypes.data,
                     active_max, learn_from)
    out = np.zeros(n, dtype=np.int8)
    res = LearnedResult()
    _check(lib().gdi_anneal_learned(h, ctypes.byref(s), ctypes.c_uint64(seed), _ptr(w), ctypes.byref(cfg), _ptr(out),
                                    ctypes.byref(res)))
    d = dict(spins=out, M=res.magnetization, cut=res.cut_weighted, result=res.as_dict())
    if mask_trace:
        d["masks"] = masks
    return d


def collect_traces(h, temps, seed: int, every: int, k_label: int, d_x: int, d_y: int, max_snapshots: int,
                   A: int = 1, B: int = 1, replica: int = 0, mode: int = BAL_GATED) -> int:
    """gdi_collect_traces into device buffers (d_x: max_snapshots*n*8 bf16, d_y: max_snapshots*n bytes)."""
    s, T = _schedule(temps, A, B, replica, mode, 0, None, None, None)
    cnt = ctypes.c_uint32()
    _check(lib().gdi_collect_traces(h, ctypes.byref(s), ctypes.c_uint64(seed), every, k_label, ctypes.c_void_p(d_x),
                                    ctypes.c_void_p(d_y), max_snapshots, ctypes.byref(cnt)))
    return cnt.value


def mlp_train(d_x: int, d_y: int, n: int, weights, epochs: int, batch: int, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, seed: int = 0, stream: int | None = None) -> tuple:
    """gdi_mlp_train: returns (trained flat weights, per-epoch mean loss)."""
    w = _weights(weights).copy()
    cfg = TrainCfg(epochs, batch, lr, beta1, beta2, eps, seed)
    losses = np.zeros(epochs, dtype=np.float32)
    _check(lib().gdi_mlp_train(ctypes.c_void_p(d_x), ctypes.c_void_p(d_y), ctypes.c_uint64(n), _ptr(w),
                               ctypes.byref(cfg), _ptr(losses), stream))
    return w, losses


def mlp_forward(weights, d_x: int, n: int, d_logits: int, stream: int | None = None):
    _check(lib().gdi_mlp_forward(_ptr(_weights(weights)), ctypes.c_void_p(d_x), n, ctypes.c_void_p(d_logits), stream))


def mlp_gradient(weights, d_x: int, d_y: int, n: int, stream: int | None = None) -> tuple:
    """gdi_mlp_gradient: (flat gradient, mean loss)."""
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_float()
    _check(lib().gdi_mlp_gradient(_ptr(_weights(weights)), ctypes.c_void_p(d_x), ctypes.c_void_p(d_y), n, _ptr(g),
                                  ctypes.byref(loss), stream))
    return g, loss.value


class Annealer:
    """Owns one gdi_graph handle for a graph with fields n, row_ptr, col, w."""

    def __init__(self, graph):
        self.n = int(graph.n)
        self.h = create(graph.row_ptr, graph.col, graph.w, self.n)
        self.info = get_info(self.h)

    def close(self):
        if self.h:
            destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def anneal(self, temps, seed, **kw) -> dict:
        return anneal(self.h, self.n, temps, seed, **kw)

    def anneal_dev(self, temps, seed, d_spins_out, **kw):
        anneal_dev(self.h, temps, seed, d_spins_out, **kw)

    def cut(self, spins):
        return cut(self.h, spins)

    def cut_dev(self, d_spins: int):
        return cut_dev(self.h, d_spins)

    def cut_dev_noalloc(self, d_spins: int, d_out: int):
        cut_dev_noalloc(self.h, d_spins, d_out)

    def result(self) -> Result:
        return last_result(self.h)

    def tune(self, **kw):
        set_tuning(self.h, **kw)

    def autotune(self, temps, seed, probe_sweeps=0, use_cache=False, **kw) -> tuple:
        return autotune(self.h, temps, seed, probe_sweeps, use_cache, **kw)

    def set_stream(self, stream_ptr):
        set_stream(self.h, stream_ptr)

    def anneal_learned(self, temps, seed, k_full, **kw) -> dict:
        return anneal_learned(self.h, self.n, temps, seed, k_full, **kw)

    def collect_traces(self, temps, seed, every, k_label, d_x, d_y, max_snapshots, **kw) -> int:
        return collect_traces(self.h, temps, seed, every, k_label, d_x, d_y, max_snapshots, **kw)

    def colouring(self):
        return get_colouring(self.h, self.n, self.info.n_colours)
