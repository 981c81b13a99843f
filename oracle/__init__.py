"""CPU oracle for fingerprint-filtered approximate dictionary matching.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything in this package, and this package imports nothing from
the product library.

The arithmetic lives in ``oracle.c`` (plain C, built into ``liboracle.so`` by
``oracle.build``); this module is argument marshalling over ctypes.  What each
function computes, and the passage of the paper it follows:

* ``ham`` / ``lev``: Hamming and Levenshtein distance (Section 1), Hamming
  infinite (``None``) when lengths differ (proof of Theorem 1).
* ``match``: every (query, word) pair compared exactly, result sorted by
  (query, word) (the dictionary-matching problem of Section 1).
* ``select_symbols``: common / rare / mixed symbol sets (Section 3).
* ``fingerprints``: occurrence, occurrence-halved, count, position
  constructions (Section 3.2), and hashed bigram occurrence (``QGRAM``, the
  q-gram direction of the future work in Section 5), and occurrence + count
  combined in one word (``COMBO``, F_D = the larger part's).
* ``fd``: fingerprint distance F_D (Section 3.3); a pair is rejected when
  ceil(F_D/2) > k (Eq. 1), i.e. survives when F_D <= 2k.
* ``filter_stats``: examined / surviving pair counts under Eq. 1.
* ``excess`` / ``filter_stats_asym``: the one-directional halves of F_D and
  the bound max(excess(q, w), excess(w, q)) <= k built from them -- an
  extension beyond the paper (it follows from the per-edit argument of
  Theorem 1 applied to each direction separately), not one of its filters.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HAM, LEV = 0, 1
OCC, COUNT, POS, OCCH, QGRAM, COMBO = 0, 1, 2, 3, 4, 5
COMMON, RARE, MIXED = 0, 1, 2
NONE = 0xFF
INF = 0xFFFFFFFF

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.orc_ham.restype = ctypes.c_uint32
    lib.orc_ham.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32]
    lib.orc_lev.restype = ctypes.c_uint32
    lib.orc_lev.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32]
    lib.orc_match.restype = ctypes.c_int
    lib.orc_match.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32, ctypes.c_int,
                              ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                              ctypes.POINTER(u32p), u64p]
    lib.orc_pair_dist.restype = ctypes.c_int
    lib.orc_pair_dist.argtypes = [u8p, u64p, u8p, u64p, u32p, ctypes.c_uint64, ctypes.c_int, u32p]
    lib.orc_free.restype = None
    lib.orc_free.argtypes = [ctypes.c_void_p]
    lib.orc_host_threads.restype = ctypes.c_uint32
    lib.orc_host_threads.argtypes = []
    lib.orc_num_fields.restype = ctypes.c_int
    lib.orc_num_fields.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.orc_histogram.restype = None
    lib.orc_histogram.argtypes = [u8p, u64p, ctypes.c_uint32, u64p]
    lib.orc_select_symbols.restype = ctypes.c_int
    lib.orc_select_symbols.argtypes = [u64p, ctypes.c_int, ctypes.c_uint32, ctypes.c_int, u8p]
    lib.orc_fp.restype = ctypes.c_uint32
    lib.orc_fp.argtypes = [u8p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, u8p]
    lib.orc_check_map.restype = ctypes.c_int
    lib.orc_check_map.argtypes = [u8p, ctypes.c_int, ctypes.c_uint32]
    lib.orc_fp_many.restype = ctypes.c_int
    lib.orc_fp_many.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, u8p, u32p]
    lib.orc_fd.restype = ctypes.c_uint32
    lib.orc_fd.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_int]
    lib.orc_fd_many.restype = None
    lib.orc_fd_many.argtypes = [u32p, u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_int, u32p]
    lib.orc_filter_stats.restype = ctypes.c_int
    lib.orc_filter_stats.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32, ctypes.c_int,
                                     ctypes.c_uint32, u8p, ctypes.c_int, ctypes.c_uint32, u64p]
    lib.orc_threshold.restype = ctypes.c_uint32
    lib.orc_threshold.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.orc_excess.restype = ctypes.c_uint32
    lib.orc_excess.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32]
    lib.orc_excess_many.restype = None
    lib.orc_excess_many.argtypes = [u32p, u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, u32p]
    lib.orc_filter_stats_asym.restype = ctypes.c_int
    lib.orc_filter_stats_asym.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u64p, ctypes.c_uint32, ctypes.c_int,
                                          ctypes.c_uint32, u8p, ctypes.c_int, ctypes.c_uint32, u64p]
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _bytes(s) -> np.ndarray:
    if isinstance(s, str):
        s = s.encode("latin-1")
    return np.frombuffer(bytes(s) + b"\0", dtype=np.uint8)


def _csr(strings):
    """(bytes, offsets) numpy pair from a CSR tuple or a list of byte strings."""
    if isinstance(strings, tuple):
        b, o = strings
        b = np.ascontiguousarray(b, dtype=np.uint8)
        if b.size == 0:
            b = np.zeros(1, dtype=np.uint8)
        return b, np.ascontiguousarray(o, dtype=np.uint64)
    items = [s.encode("latin-1") if isinstance(s, str) else bytes(s) for s in strings]
    offs = np.zeros(len(items) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(s) for s in items], dtype=np.uint64)
    b = np.frombuffer(b"".join(items) + b"\0", dtype=np.uint8).copy()
    return b, offs


def host_threads() -> int:
    return int(_load().orc_host_threads())


def ham(a, b):
    """Hamming distance, or None when the lengths differ."""
    x, y = _bytes(a), _bytes(b)
    d = _load().orc_ham(_ptr(x, ctypes.c_uint8), x.size - 1, _ptr(y, ctypes.c_uint8), y.size - 1)
    return None if d == INF else int(d)


def lev(a, b) -> int:
    x, y = _bytes(a), _bytes(b)
    return int(_load().orc_lev(_ptr(x, ctypes.c_uint8), x.size - 1, _ptr(y, ctypes.c_uint8), y.size - 1))


def match(dictionary, queries, metric: int, k: int, threads: int = 0, length_pruned: bool = False) -> np.ndarray:
    """All (query, word, dist) with dist <= k as an (n, 3) uint32 array sorted
    by (query, word).  ``length_pruned`` skips Lev pairs with |m-n| > k (exact
    because Lev >= |m-n|); it is off by default."""
    lib = _load()
    db, do = _csr(dictionary)
    qb, qo = _csr(queries)
    out = ctypes.POINTER(ctypes.c_uint32)()
    n = ctypes.c_uint64(0)
    rc = lib.orc_match(_ptr(db, ctypes.c_uint8), _ptr(do, ctypes.c_uint64), do.size - 1,
                       _ptr(qb, ctypes.c_uint8), _ptr(qo, ctypes.c_uint64), qo.size - 1,
                       metric, k, threads, 1 if length_pruned else 0, ctypes.byref(out), ctypes.byref(n))
    if rc != 0:
        raise ValueError("oracle match failed (bad metric or a string longer than 255)")
    if n.value == 0:
        return np.zeros((0, 3), dtype=np.uint32)
    res = np.ctypeslib.as_array(out, shape=(n.value * 3,)).copy().reshape(-1, 3)
    lib.orc_free(out)
    return res


def pair_dist(dictionary, queries, pairs: np.ndarray, metric: int) -> np.ndarray:
    """Exact distance of each (query, word) pair; INF for infinite Hamming."""
    lib = _load()
    db, do = _csr(dictionary)
    qb, qo = _csr(queries)
    p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros(p.shape[0], dtype=np.uint32)
    rc = lib.orc_pair_dist(_ptr(db, ctypes.c_uint8), _ptr(do, ctypes.c_uint64), _ptr(qb, ctypes.c_uint8),
                           _ptr(qo, ctypes.c_uint64), _ptr(p, ctypes.c_uint32), p.shape[0], metric,
                           _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("oracle pair_dist failed")
    return out


def num_fields(variant: int, bits: int) -> int:
    return int(_load().orc_num_fields(variant, bits))


def histogram(strings) -> np.ndarray:
    b, o = _csr(strings)
    h = np.zeros(256, dtype=np.uint64)
    _load().orc_histogram(_ptr(b, ctypes.c_uint8), _ptr(o, ctypes.c_uint64), o.size - 1, _ptr(h, ctypes.c_uint64))
    return h


def select_symbols(hist: np.ndarray, variant: int, bits: int, symset: int) -> np.ndarray:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    m = np.zeros(256, dtype=np.uint8)
    if _load().orc_select_symbols(_ptr(h, ctypes.c_uint64), variant, bits, symset, _ptr(m, ctypes.c_uint8)) < 0:
        raise ValueError("bad variant/bits/symbol set")
    return m


def check_map(mp: np.ndarray, variant: int, bits: int) -> bool:
    m = np.ascontiguousarray(mp, dtype=np.uint8)
    return _load().orc_check_map(_ptr(m, ctypes.c_uint8), variant, bits) == 0


def fingerprint(s, variant: int, bits: int, mp: np.ndarray) -> int:
    x = _bytes(s)
    m = np.ascontiguousarray(mp, dtype=np.uint8)
    if not check_map(m, variant, bits):
        raise ValueError("bad symbol map")
    return int(_load().orc_fp(_ptr(x, ctypes.c_uint8), x.size - 1, variant, bits, _ptr(m, ctypes.c_uint8)))


def fingerprints(strings, variant: int, bits: int, mp: np.ndarray) -> np.ndarray:
    b, o = _csr(strings)
    m = np.ascontiguousarray(mp, dtype=np.uint8)
    out = np.zeros(max(o.size - 1, 1), dtype=np.uint32)
    rc = _load().orc_fp_many(_ptr(b, ctypes.c_uint8), _ptr(o, ctypes.c_uint64), o.size - 1, variant, bits,
                             _ptr(m, ctypes.c_uint8), _ptr(out, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("bad symbol map")
    return out[: o.size - 1]


def fd(a, b, variant: int, bits: int, literal: bool = False):
    """F_D of fingerprint pairs; scalars or equal-length arrays."""
    if np.isscalar(a) and np.isscalar(b):
        return int(_load().orc_fd(int(a), int(b), variant, bits, 1 if literal else 0))
    x = np.ascontiguousarray(a, dtype=np.uint32)
    y = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.zeros(x.size, dtype=np.uint32)
    _load().orc_fd_many(_ptr(x, ctypes.c_uint32), _ptr(y, ctypes.c_uint32), x.size, variant, bits,
                        1 if literal else 0, _ptr(out, ctypes.c_uint32))
    return out


def threshold(variant: int, k: int) -> int:
    """Largest F_D of a pair within distance k: 2k (Eq. 1), 4k for bigrams."""
    return int(_load().orc_threshold(variant, k))


def excess(a, b, variant: int, bits: int):
    """Excess of fingerprint a over b (occ: fields set in a only; count: sum of
    positive count differences); scalars or equal-length arrays."""
    if np.isscalar(a) and np.isscalar(b):
        return int(_load().orc_excess(int(a), int(b), variant, bits))
    x = np.ascontiguousarray(a, dtype=np.uint32)
    y = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.zeros(x.size, dtype=np.uint32)
    _load().orc_excess_many(_ptr(x, ctypes.c_uint32), _ptr(y, ctypes.c_uint32), x.size, variant, bits,
                            _ptr(out, ctypes.c_uint32))
    return out


def filter_stats_asym(dictionary, queries, variant: int, bits: int, mp: np.ndarray, metric: int, k: int):
    """(examined, survivors) over all pairs under the asymmetric bound
    max(excess(q, w), excess(w, q)) <= k."""
    db, do = _csr(dictionary)
    qb, qo = _csr(queries)
    m = np.ascontiguousarray(mp, dtype=np.uint8)
    c = np.zeros(2, dtype=np.uint64)
    rc = _load().orc_filter_stats_asym(_ptr(db, ctypes.c_uint8), _ptr(do, ctypes.c_uint64), do.size - 1,
                                       _ptr(qb, ctypes.c_uint8), _ptr(qo, ctypes.c_uint64), qo.size - 1, variant,
                                       bits, _ptr(m, ctypes.c_uint8), metric, k, _ptr(c, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad symbol map or variant")
    return int(c[0]), int(c[1])


def filter_stats(dictionary, queries, variant: int, bits: int, mp: np.ndarray, metric: int, k: int):
    """(examined, survivors, survivors_literal) over all pairs."""
    db, do = _csr(dictionary)
    qb, qo = _csr(queries)
    m = np.ascontiguousarray(mp, dtype=np.uint8)
    c = np.zeros(3, dtype=np.uint64)
    rc = _load().orc_filter_stats(_ptr(db, ctypes.c_uint8), _ptr(do, ctypes.c_uint64), do.size - 1,
                                  _ptr(qb, ctypes.c_uint8), _ptr(qo, ctypes.c_uint64), qo.size - 1, variant, bits,
                                  _ptr(m, ctypes.c_uint8), metric, k, _ptr(c, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad symbol map")
    return int(c[0]), int(c[1]), int(c[2])
