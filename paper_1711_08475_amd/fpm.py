"""ctypes binding of libfpm (include/fpm.h).

Argument marshalling only: every step of matching runs in the library's HIP
kernels.  The functions keep the C names.  Host-buffer entry points take
strings in CSR form, ``(bytes uint8[total], offsets uint64[n+1])``; the plan
entry points take device pointers (for example ``tensor.data_ptr()`` of torch
CUDA tensors) and a HIP stream handle.

Loading fails loudly when ``libfpm.so`` has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpm.so")

FPM_OK, FPM_EINVAL, FPM_EUNSUPPORTED, FPM_ENOMEM, FPM_EDEVICE = 0, -1, -2, -3, -4
FPM_OCC, FPM_COUNT, FPM_POS, FPM_OCCH, FPM_QGRAM, FPM_COMBO = 0, 1, 2, 3, 4, 5
FPM_HAM, FPM_LEV = 0, 1
FPM_COMMON, FPM_RARE, FPM_MIXED, FPM_CUSTOM = 0, 1, 2, 3
FPM_SCHED_PLAIN, FPM_SCHED_BATCHED, FPM_SCHED_BRUTE = 0, 1, 2

VARIANTS = {"occ": FPM_OCC, "count": FPM_COUNT, "pos": FPM_POS, "occh": FPM_OCCH, "qgram": FPM_QGRAM,
            "combo": FPM_COMBO}
METRICS = {"ham": FPM_HAM, "lev": FPM_LEV}
SYMBOLS = {"common": FPM_COMMON, "rare": FPM_RARE, "mixed": FPM_MIXED, "custom": FPM_CUSTOM}
FPM_BOUND_FD, FPM_BOUND_ASYM = 0, 1
BOUNDS = {"fd": FPM_BOUND_FD, "asym": FPM_BOUND_ASYM}
FPM_UNIT_AUTO, FPM_UNIT_VALU, FPM_UNIT_MATRIX = 0, 1, 2
UNITS = {"auto": FPM_UNIT_AUTO, "valu": FPM_UNIT_VALU, "matrix": FPM_UNIT_MATRIX}
FPM_PRUNE_OFF, FPM_PRUNE_ON = 0, 1
PRUNES = {"off": FPM_PRUNE_OFF, "on": FPM_PRUNE_ON}

# every symbol include/fpm.h declares
EXPORTS = [
    "fpm_last_error", "fpm_free", "fpm_num_fields", "fpm_select_symbols", "fpm_build_fingerprints",
    "fpm_index_destroy", "fpm_get_fingerprints", "fpm_get_map", "fpm_index_info", "fpm_fingerprints",
    "fpm_match", "fpm_filter_pairs", "fpm_verify_pairs", "fpm_plan_create", "fpm_plan_run", "fpm_plan_result",
    "fpm_plan_copy_matches", "fpm_plan_destroy", "fpm_autotune", "fpm_plan_kernel_ms", "fpm_index_build_ms",
    "fpm_set_device_memory_limit", "fpm_device_memory_in_use", "fpm_match_noalloc",
]
# every symbol include/fpm_learn.h declares
LEARN_EXPORTS = ["fpm_learn_grouping", "fpm_learn_step"]
# every symbol include/fpm_peak.h declares
PEAK_EXPORTS = ["fpm_measure_peaks"]


class FpmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fpm status {status}: {msg}")
        self.status = status


class Hit(ctypes.Structure):
    _fields_ = [("query", ctypes.c_uint32), ("word", ctypes.c_uint32), ("dist", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("pairs_logical", ctypes.c_uint64), ("pairs_examined", ctypes.c_uint64),
                ("survivors", ctypes.c_uint64), ("matches", ctypes.c_uint64), ("verify_cells", ctypes.c_uint64),
                ("pairs_filtered", ctypes.c_uint64), ("ms", ctypes.c_float), ("work_items", ctypes.c_uint32),
                ("filter_unit", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_uint32), ("queries_per_item", ctypes.c_uint32), ("slab", ctypes.c_uint32),
                ("bucket_order", ctypes.c_uint32), ("use_graph", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("match_capacity", ctypes.c_uint32), ("time_kernel", ctypes.c_uint32),
                ("tail_split", ctypes.c_uint32), ("bound", ctypes.c_uint32), ("filter_unit", ctypes.c_uint32),
                ("pop_prune", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 4)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Peaks(ctypes.Structure):
    _fields_ = [("int_valu_ops_per_s", ctypes.c_double), ("int8_matrix_ops_per_s", ctypes.c_double),
                ("valu_ops", ctypes.c_uint64), ("matrix_ops", ctypes.c_uint64), ("valu_ms", ctypes.c_float),
                ("matrix_ms", ctypes.c_float), ("compute_units", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class LearnConfig(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_uint32), ("k", ctypes.c_uint32), ("hidden", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("margin", ctypes.c_float), ("beta", ctypes.c_float), ("entropy_weight", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class LearnReport(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_uint32), ("d_in", ctypes.c_uint32), ("n_params", ctypes.c_uint32),
                ("steps", ctypes.c_uint32), ("train_pairs", ctypes.c_uint64), ("first_loss", ctypes.c_float),
                ("final_loss", ctypes.c_float), ("final_entropy", ctypes.c_float), ("expected_fd", ctypes.c_float),
                ("ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def options(**kw) -> Options:
    o = Options()
    names = {f for f, _ in Options._fields_ if f != "reserved"}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}")
        if k == "bound":
            v = _code(BOUNDS, v)
        if k == "filter_unit":
            v = _code(UNITS, v)
        if k == "pop_prune":
            v = _code(PRUNES, v)
        setattr(o, k, v)
    return o


_lib = None
u8p = ctypes.POINTER(ctypes.c_uint8)
u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)
vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build()); no fallback exists")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "fpm_last_error": (ctypes.c_char_p, []),
        "fpm_free": (None, [vp]),
        "fpm_num_fields": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32]),
        "fpm_select_symbols": (ctypes.c_int, [u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                              ctypes.c_int, u8p]),
        "fpm_build_fingerprints": (ctypes.c_int, [u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                                  ctypes.c_int, u8p, ctypes.POINTER(vp)]),
        "fpm_index_destroy": (None, [vp]),
        "fpm_get_fingerprints": (ctypes.c_int, [vp, u32p]),
        "fpm_get_map": (ctypes.c_int, [vp, u8p]),
        "fpm_index_info": (ctypes.c_int, [vp, u32p, u32p, u32p]),
        "fpm_index_build_ms": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
        "fpm_set_device_memory_limit": (ctypes.c_int, [ctypes.c_uint64]),
        "fpm_device_memory_in_use": (ctypes.c_int, [u64p]),
        "fpm_fingerprints": (ctypes.c_int, [vp, u8p, u64p, ctypes.c_uint32, u32p]),
        "fpm_match": (ctypes.c_int, [vp, u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                     ctypes.POINTER(Options), ctypes.POINTER(ctypes.POINTER(Hit)), u64p,
                                     ctypes.POINTER(Stats)]),
        "fpm_filter_pairs": (ctypes.c_int, [vp, u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                            ctypes.POINTER(u32p), u64p]),
        "fpm_verify_pairs": (ctypes.c_int, [vp, u8p, u64p, ctypes.c_uint32, u32p, ctypes.c_uint64, ctypes.c_int,
                                            ctypes.c_uint32, u32p]),
        "fpm_plan_create": (ctypes.c_int, [vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                           ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]),
        "fpm_plan_run": (ctypes.c_int, [vp, vp, vp, ctypes.c_uint32]),
        "fpm_plan_result": (ctypes.c_int, [vp, ctypes.POINTER(vp), u64p, ctypes.POINTER(Stats)]),
        "fpm_plan_copy_matches": (ctypes.c_int, [vp, vp, ctypes.c_uint64, u64p]),
        "fpm_plan_destroy": (None, [vp]),
        "fpm_match_noalloc": (ctypes.c_int, [vp, vp, vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                             ctypes.c_uint32, ctypes.POINTER(Options), vp, vp, ctypes.c_uint64, u64p,
                                             ctypes.POINTER(Stats)]),
        "fpm_plan_kernel_ms": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_uint32, u32p]),
        "fpm_autotune": (ctypes.c_int, [vp, vp, vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Options),
                                        ctypes.POINTER(ctypes.c_float), ctypes.c_uint32, u32p]),
    }
    fp = ctypes.POINTER(ctypes.c_float)
    sig["fpm_learn_grouping"] = (ctypes.c_int, [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32, u32p, u8p,
                                                ctypes.c_uint64, ctypes.POINTER(LearnConfig), u8p,
                                                ctypes.POINTER(LearnReport)])
    sig["fpm_learn_step"] = (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, fp, fp, u64p, u64p, ctypes.c_uint64, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, fp, fp, fp])
    sig["fpm_measure_peaks"] = (ctypes.c_int, [ctypes.POINTER(Peaks)])
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int):
    if st != FPM_OK:
        raise FpmError(st, lib().fpm_last_error().decode(errors="replace"))


def _csr(csr):
    b, o = csr
    b = np.ascontiguousarray(b, dtype=np.uint8)
    if b.size == 0:
        b = np.zeros(1, dtype=np.uint8)
    o = np.ascontiguousarray(o, dtype=np.uint64)
    return b, o


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


# ------------------------------------------------------------------- index

def fpm_num_fields(variant, bits: int) -> int:
    return int(lib().fpm_num_fields(_code(VARIANTS, variant), bits))


def fpm_select_symbols(csr, variant, bits: int, symbols) -> np.ndarray:
    b, o = _csr(csr)
    m = np.zeros(256, dtype=np.uint8)
    _check(lib().fpm_select_symbols(_p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                                    _code(VARIANTS, variant), bits, _code(SYMBOLS, symbols), _p(m, ctypes.c_uint8)))
    return m


class Index:
    """Owns an fpm_index handle."""

    def __init__(self, handle, n_words: int, variant: int, bits: int):
        self.handle = handle
        self.n_words, self.variant, self.bits = n_words, variant, bits

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fpm_index_destroy(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle


def fpm_build_fingerprints(csr, variant="occ", bits: int = 16, symbols="common", custom_map=None) -> Index:
    b, o = _csr(csr)
    out = vp()
    cm = None
    if custom_map is not None:
        cm = np.ascontiguousarray(custom_map, dtype=np.uint8)
        symbols = FPM_CUSTOM
    _check(lib().fpm_build_fingerprints(_p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                                        _code(VARIANTS, variant), bits, _code(SYMBOLS, symbols),
                                        _p(cm, ctypes.c_uint8) if cm is not None else None, ctypes.byref(out)))
    return Index(out, o.size - 1, _code(VARIANTS, variant), bits)


def fpm_get_fingerprints(ix: Index) -> np.ndarray:
    out = np.zeros(max(ix.n_words, 1), dtype=np.uint32)
    _check(lib().fpm_get_fingerprints(ix.handle, _p(out, ctypes.c_uint32)))
    return out[: ix.n_words]


def fpm_get_map(ix: Index) -> np.ndarray:
    m = np.zeros(256, dtype=np.uint8)
    _check(lib().fpm_get_map(ix.handle, _p(m, ctypes.c_uint8)))
    return m


def fpm_index_info(ix: Index):
    n, v, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().fpm_index_info(ix.handle, ctypes.byref(n), ctypes.byref(v), ctypes.byref(b)))
    return n.value, v.value, b.value


def fpm_index_build_ms(ix: Index):
    """(total, layout) device ms of the index build."""
    t, l = ctypes.c_float(), ctypes.c_float()
    _check(lib().fpm_index_build_ms(ix.handle, ctypes.byref(t), ctypes.byref(l)))
    return t.value, l.value


def fpm_set_device_memory_limit(max_bytes: int):
    _check(lib().fpm_set_device_memory_limit(max_bytes))


def fpm_device_memory_in_use() -> int:
    n = ctypes.c_uint64()
    _check(lib().fpm_device_memory_in_use(ctypes.byref(n)))
    return n.value


def fpm_fingerprints(ix: Index, csr) -> np.ndarray:
    b, o = _csr(csr)
    out = np.zeros(max(o.size - 1, 1), dtype=np.uint32)
    _check(lib().fpm_fingerprints(ix.handle, _p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                                  _p(out, ctypes.c_uint32)))
    return out[: o.size - 1]


# ------------------------------------------------------------------ matching

def fpm_match(ix: Index, queries, metric="lev", k: int = 1, opts: Options | None = None, with_stats=False):
    """Sorted (n, 3) uint32 array of (query, word, dist)."""
    b, o = _csr(queries)
    out = ctypes.POINTER(Hit)()
    n = ctypes.c_uint64()
    st = Stats()
    _check(lib().fpm_match(ix.handle, _p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                           _code(METRICS, metric), k, ctypes.byref(opts) if opts is not None else None,
                           ctypes.byref(out), ctypes.byref(n), ctypes.byref(st)))
    if n.value:
        res = np.ctypeslib.as_array(ctypes.cast(out, u32p), shape=(n.value * 3,)).copy().reshape(-1, 3)
        lib().fpm_free(ctypes.cast(out, vp))
    else:
        res = np.zeros((0, 3), dtype=np.uint32)
    return (res, st.as_dict()) if with_stats else res


def fpm_filter_pairs(ix: Index, queries, metric="lev", k: int = 1) -> np.ndarray:
    b, o = _csr(queries)
    out = u32p()
    n = ctypes.c_uint64()
    _check(lib().fpm_filter_pairs(ix.handle, _p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                                  _code(METRICS, metric), k, ctypes.byref(out), ctypes.byref(n)))
    if not n.value:
        return np.zeros((0, 2), dtype=np.uint32)
    res = np.ctypeslib.as_array(out, shape=(n.value * 2,)).copy().reshape(-1, 2)
    lib().fpm_free(ctypes.cast(out, vp))
    return res


def fpm_verify_pairs(ix: Index, queries, pairs: np.ndarray, metric="lev", k: int = 1) -> np.ndarray:
    b, o = _csr(queries)
    p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros(max(p.shape[0], 1), dtype=np.uint32)
    _check(lib().fpm_verify_pairs(ix.handle, _p(b, ctypes.c_uint8), _p(o, ctypes.c_uint64), o.size - 1,
                                  _p(p, ctypes.c_uint32), p.shape[0], _code(METRICS, metric), k,
                                  _p(out, ctypes.c_uint32)))
    return out[: p.shape[0]]


# --------------------------------------------------------------------- plans

class Plan:
    def __init__(self, handle, ix: Index):
        self.handle, self.ix = handle, ix  # keeps the index alive

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fpm_plan_destroy(self.handle)
            self.handle = None


def fpm_plan_create(ix: Index, max_queries: int, max_query_bytes: int, metric="lev", k: int = 1,
                    opts: Options | None = None, stream: int | None = None) -> Plan:
    out = vp()
    _check(lib().fpm_plan_create(ix.handle, max_queries, max_query_bytes, _code(METRICS, metric), k,
                                 ctypes.byref(opts) if opts is not None else None,
                                 vp(stream) if stream else None, ctypes.byref(out)))
    return Plan(out, ix)


def fpm_plan_run(plan: Plan, d_qbytes: int, d_qoffsets: int, n_queries: int):
    _check(lib().fpm_plan_run(plan.handle, vp(d_qbytes), vp(d_qoffsets), n_queries))


def fpm_plan_result(plan: Plan):
    """(device pointer of the matches, count, stats dict)."""
    dm = vp()
    n = ctypes.c_uint64()
    st = Stats()
    _check(lib().fpm_plan_result(plan.handle, ctypes.byref(dm), ctypes.byref(n), ctypes.byref(st)))
    return dm.value, n.value, st.as_dict()


def fpm_plan_copy_matches(plan: Plan) -> np.ndarray:
    _, n, _ = fpm_plan_result(plan)
    out = np.zeros((max(n, 1), 3), dtype=np.uint32)
    got = ctypes.c_uint64()
    _check(lib().fpm_plan_copy_matches(plan.handle, out.ctypes.data_as(vp), n, ctypes.byref(got)))
    return out[: got.value]


def fpm_plan_kernel_ms(plan: Plan, max_runs: int = 256) -> np.ndarray:
    """Match-kernel durations (ms) of the last runs of a time_kernel plan."""
    out = np.zeros(max(max_runs, 1), dtype=np.float32)
    n = ctypes.c_uint32()
    _check(lib().fpm_plan_kernel_ms(plan.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), max_runs,
                                    ctypes.byref(n)))
    return out[: n.value]


NOALLOC_MAX_QUERIES, NOALLOC_MAX_QUERY_BYTES, NOALLOC_MAX_MATCHES = 65536, 4 << 20, 1 << 20


def fpm_match_noalloc(ix: Index, d_qbytes: int, d_qoffsets: int, n_queries: int, query_bytes: int, d_out: int,
                      out_cap: int, metric="lev", k: int = 1, opts: Options | None = None, stream: int | None = None):
    """Allocation-free match into the caller's device array d_out (out_cap
    fpm_hit entries): (number of matches, stats dict)."""
    n = ctypes.c_uint64()
    st = Stats()
    rc = lib().fpm_match_noalloc(ix.handle, vp(d_qbytes) if d_qbytes else None,
                                 vp(d_qoffsets) if d_qoffsets else None, n_queries, query_bytes,
                                 _code(METRICS, metric), k, ctypes.byref(opts) if opts is not None else None,
                                 vp(stream) if stream else None, vp(d_out) if d_out else None, out_cap,
                                 ctypes.byref(n), ctypes.byref(st))
    if rc != FPM_OK:
        err = FpmError(rc, lib().fpm_last_error().decode(errors="replace"))
        err.n_out = n.value  # the match count, when the list did not fit
        raise err
    return n.value, st.as_dict()


def fpm_autotune(ix: Index, d_qbytes: int, d_qoffsets: int, n_queries: int, query_bytes: int, metric="lev",
                 k: int = 1, repeats: int = 3, base: Options | None = None):
    best = base if base is not None else Options()
    tim = (ctypes.c_float * (5 * 128))()
    nt = ctypes.c_uint32()
    _check(lib().fpm_autotune(ix.handle, vp(d_qbytes), vp(d_qoffsets), n_queries, query_bytes,
                              _code(METRICS, metric), k, repeats, ctypes.byref(best), tim, 128, ctypes.byref(nt)))
    rows = [tuple(tim[5 * i:5 * i + 5]) for i in range(nt.value)]
    return best, rows


# ------------------------------------------------------------ learned grouping

def fpm_learn_grouping(dictionary, queries, pairs: np.ndarray, is_match: np.ndarray, cfg: LearnConfig):
    """(map uint8[256], report dict)."""
    db, do = _csr(dictionary)
    qb, qo = _csr(queries)
    p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    m = np.ascontiguousarray(is_match, dtype=np.uint8)
    if p.shape[0] == 0:
        p = np.zeros((1, 2), dtype=np.uint32)[:0]
    out = np.zeros(256, dtype=np.uint8)
    rep = LearnReport()
    _check(lib().fpm_learn_grouping(_p(db, ctypes.c_uint8), _p(do, ctypes.c_uint64), do.size - 1,
                                    _p(qb, ctypes.c_uint8), _p(qo, ctypes.c_uint64), qo.size - 1,
                                    _p(np.ascontiguousarray(p), ctypes.c_uint32), _p(m, ctypes.c_uint8), p.shape[0],
                                    ctypes.byref(cfg), _p(out, ctypes.c_uint8), ctypes.byref(rep)))
    return out, rep.as_dict()


def fpm_learn_step(X, params, hidden: int, bits: int, k: int, masks_a, masks_b, margin: float, beta: float,
                   entropy_weight: float):
    """One GPU forward/backward: (P, [pair loss, entropy, mean E], grads)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    prm = np.ascontiguousarray(params, dtype=np.float32)
    ma = np.ascontiguousarray(masks_a, dtype=np.uint64).reshape(-1, 2)
    mb = np.ascontiguousarray(masks_b, dtype=np.uint64).reshape(-1, 2)
    sigma, d_in = X.shape
    P = np.zeros((sigma, bits + 1), dtype=np.float32)
    loss = np.zeros(3, dtype=np.float32)
    g = np.zeros_like(prm)
    fp = ctypes.c_float
    _check(lib().fpm_learn_step(sigma, d_in, hidden, bits, k, _p(X, fp), _p(prm, fp), _p(ma, ctypes.c_uint64),
                                _p(mb, ctypes.c_uint64), ma.shape[0], margin, beta, entropy_weight, _p(P, fp),
                                _p(loss, fp), _p(g, fp)))
    return P, loss, g


# ------------------------------------------------------------ peak probes

def fpm_measure_peaks() -> dict:
    """Measured int-VALU and int8 matrix-core peaks of the current device."""
    out = Peaks()
    _check(lib().fpm_measure_peaks(ctypes.byref(out)))
    return out.as_dict()
