"""CPU oracle of the k-mer counting path.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The product library
never imports, links or runs anything in this directory.

``kc_oracle.c`` (plain C, built with gcc) holds the reference computation;
``brute.py`` is a second, pure-Python reading of the same definitions used to
pin the C code on tiny inputs.  Each function names the passage of the paper it
follows in the C source header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U64P = ctypes.POINTER(ctypes.c_uint64)
U32P = ctypes.POINTER(ctypes.c_uint32)
U8P = ctypes.POINTER(ctypes.c_uint8)
RANGE_CB = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, U64P, U32P, ctypes.c_uint64)


class OrParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("n_counters", ctypes.c_uint32),
                ("min_count", ctypes.c_uint32), ("m_log2", ctypes.c_uint32),
                ("h", ctypes.c_uint32), ("block_log2", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


class OrStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_valid", "n_distinct", "n_pass", "entries", "sum_counts", "fp_singletons",
        "b1_pop", "b2_pop")]


class OrResult(ctypes.Structure):
    _fields_ = [("st", OrStats), ("n_entries", ctypes.c_uint64), ("keys", U64P),
                ("counts", U32P), ("m_words", ctypes.c_uint64), ("b1", U64P), ("b2", U64P),
                ("n_touched", ctypes.c_uint64), ("touched", U64P), ("t1", U64P), ("t2", U64P)]


def build(force: bool = True) -> str:
    """Compile kc_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(OrParams)
        lib.or_mix64.argtypes = [ctypes.c_uint64]
        lib.or_mix64.restype = ctypes.c_uint64
        lib.or_count.argtypes = [P, U8P, U64P, ctypes.c_uint64, U8P, ctypes.c_int]
        lib.or_count.restype = ctypes.POINTER(OrResult)
        lib.or_free.argtypes = [ctypes.POINTER(OrResult)]
        lib.or_count_ranges.argtypes = [P, U8P, U64P, ctypes.c_uint64, U8P, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_int, ctypes.c_int, RANGE_CB,
                                        ctypes.c_void_p]
        lib.or_count_ranges.restype = ctypes.POINTER(OrResult)
        lib.or_enumerate.argtypes = [P, U8P, U64P, ctypes.c_uint64, U8P, U64P, ctypes.c_uint64]
        lib.or_enumerate.restype = ctypes.c_uint64
        lib.or_bloom_bits.argtypes = [P, ctypes.c_uint64, U64P]
        lib.or_bloom_bits.restype = ctypes.c_uint32
        lib.or_sample_counts.argtypes = [P, U8P, U64P, ctypes.c_uint64, U8P, U64P,
                                         ctypes.c_uint64, U32P, U64P, ctypes.c_int]
        lib.or_sample_counts.restype = ctypes.c_int
        lib.or_sample_hits.argtypes = [P, U8P, U64P, ctypes.c_uint64, U64P, ctypes.c_uint64,
                                       U32P, ctypes.c_int]
        lib.or_sample_hits.restype = ctypes.c_int
        U16PP = ctypes.POINTER(ctypes.POINTER(ctypes.c_uint16))
        lib.or_stem_items.argtypes = [ctypes.c_uint32, ctypes.c_uint32, U64P, U32P, ctypes.c_uint64,
                                      ctypes.POINTER(U64P), U16PP, U64P]
        lib.or_stem_items.restype = ctypes.c_int
        lib.or_free_ptr.argtypes = [ctypes.c_void_p]
        lib.or_filter_reads.argtypes = [ctypes.c_uint32, ctypes.c_uint32, U64P, U32P, ctypes.c_uint64,
                                        U8P, U64P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        U32P]
        lib.or_filter_reads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Params:
    k: int = 31
    n_counters: int = 1
    min_count: int = 2
    m_log2: int = 24
    h: int = 3
    block_log2: int = 19
    seed: int = 0

    def c(self) -> OrParams:
        return OrParams(self.k, self.n_counters, self.min_count, self.m_log2, self.h,
                        min(self.block_log2, self.m_log2), self.seed & ((1 << 64) - 1))


@dataclass
class Result:
    keys: np.ndarray       # uint64 [E], ascending
    counts: np.ndarray     # uint32 [E, n_counters]
    b1: np.ndarray | None  # uint64 [m/64]
    b2: np.ndarray | None
    stats: dict
    # bloom="sparse": the nonzero words of B1 (indices ascending) and both levels there
    touched: np.ndarray | None = None
    t1: np.ndarray | None = None
    t2: np.ndarray | None = None


def _arrays(bases, offsets, tags):
    bases = np.ascontiguousarray(bases, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if tags is not None:
        tags = np.ascontiguousarray(tags, dtype=np.uint8)
    return bases, offsets, tags


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def mix64(z: int) -> int:
    return int(_load().or_mix64(z & ((1 << 64) - 1)))


def _bloom_mode(want_bloom) -> int:
    return 2 if want_bloom == "sparse" else (1 if want_bloom else 0)


def count(params: Params, bases, offsets, tags=None, want_bloom=True) -> Result:
    """Full count: final table, Bloom levels and statistics.  want_bloom =
    "sparse" returns the levels as their nonzero words (Result.touched, t1,
    t2) instead of whole arrays."""
    bases, offsets, tags = _arrays(bases, offsets, tags)
    n_reads = offsets.size - 1
    p = params.c()
    r = _load().or_count(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P), n_reads,
                         _ptr(tags, U8P), _bloom_mode(want_bloom))
    return _result(r, params, want_bloom)


def count_ranges(params: Params, bases, offsets, tags=None, want_bloom=True,
                 qbits: int = 0, threads: int = 0, keep_singles: bool = True,
                 on_range=None) -> Result:
    """The same result as ``count``, by value-range passes (kc_oracle.c,
    or_count_ranges): 2^qbits ranges of the k-mer space by their top bits,
    ``threads`` of them per pass; qbits = 0 picks the smallest power of two
    that gives every thread a range.  keep_singles = False screens in a second
    round of passes instead of keeping the keys seen once.  on_range(q, keys,
    counts), when given, receives each range's final table (numpy views, valid
    during the call) in ascending order instead of the result's table."""
    bases, offsets, tags = _arrays(bases, offsets, tags)
    n_reads = offsets.size - 1
    threads = threads or _threads()
    if not qbits:
        qbits = min(2 * params.k, max(0, (threads - 1).bit_length()))
    p = params.c()
    nc = params.n_counters

    def relay(_user, q, kp, cp, n):
        keys = np.ctypeslib.as_array(kp, shape=(n,)) if n else np.zeros(0, np.uint64)
        counts = np.ctypeslib.as_array(cp, shape=(n * nc,)) if n else np.zeros(0, np.uint32)
        on_range(int(q), keys, counts.reshape(n, nc))

    cb = RANGE_CB(relay) if on_range is not None else RANGE_CB()
    r = _load().or_count_ranges(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P), n_reads,
                                _ptr(tags, U8P), _bloom_mode(want_bloom), qbits, threads,
                                1 if keep_singles else 0, cb, None)
    return _result(r, params, want_bloom)


def _result(r, params: Params, want_bloom) -> Result:
    if not r:
        raise ValueError("oracle rejected the parameters or input")
    try:
        res = r.contents
        ne = res.n_entries
        nc = params.n_counters
        keys = np.ctypeslib.as_array(res.keys, shape=(max(ne, 1),))[:ne].copy()
        counts = np.ctypeslib.as_array(res.counts, shape=(max(ne * nc, 1),))[:ne * nc].copy()
        b1 = b2 = touched = t1 = t2 = None
        if want_bloom == "sparse":
            n = res.n_touched
            touched = np.ctypeslib.as_array(res.touched, shape=(max(n, 1),))[:n].copy()
            t1 = np.ctypeslib.as_array(res.t1, shape=(max(n, 1),))[:n].copy()
            t2 = np.ctypeslib.as_array(res.t2, shape=(max(n, 1),))[:n].copy()
        elif want_bloom:
            b1 = np.ctypeslib.as_array(res.b1, shape=(res.m_words,)).copy()
            b2 = np.ctypeslib.as_array(res.b2, shape=(res.m_words,)).copy()
        st = {name: int(getattr(res.st, name)) for name, _ in OrStats._fields_}
    finally:
        _load().or_free(r)
    return Result(keys, counts.reshape(ne, nc), b1, b2, st, touched, t1, t2)


def enumerate_keys(params: Params, bases, offsets, tags=None) -> np.ndarray:
    """Canonical keys of every valid window, in read order, tagged (x << 1 | tag)."""
    bases, offsets, tags = _arrays(bases, offsets, tags)
    p = params.c()
    lib = _load()
    n = lib.or_enumerate(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P),
                         offsets.size - 1, _ptr(tags, U8P), None, 0)
    out = np.empty(max(int(n), 1), dtype=np.uint64)
    lib.or_enumerate(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P), offsets.size - 1,
                     _ptr(tags, U8P), _ptr(out, U64P), n)
    return out[:n]


def bloom_bits(params: Params, x: int) -> list[int]:
    p = params.c()
    out = np.zeros(8, dtype=np.uint64)
    n = _load().or_bloom_bits(ctypes.byref(p), x & ((1 << 64) - 1), _ptr(out, U64P))
    if n == 0:
        raise ValueError("oracle rejected the Bloom parameters")
    return [int(v) for v in out[:n]]


def stem_items(k: int, n_counters: int, keys, counts):
    """Stem items of a final table (kc_oracle.c, or_stem_items; paper Sec.
    II-A stems, Sec. III-D items of 16 normal and 16 tumour counts): returns
    (stems uint64[n] ascending, items uint16[n, 2, 16]) where items[i, t, 4a+b]
    is counter t of the k-mer a + stem + b (stem in canonical orientation)."""
    lib = _load()
    keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
    counts = np.ascontiguousarray(counts, dtype=np.uint32).reshape(-1)
    if counts.size != keys.size * n_counters:
        raise ValueError("counts must hold n_counters per key")
    sp = U64P()
    ip = ctypes.POINTER(ctypes.c_uint16)()
    n = ctypes.c_uint64(0)
    rc = lib.or_stem_items(k, n_counters, _ptr(keys, U64P), _ptr(counts, U32P), keys.size,
                           ctypes.byref(sp), ctypes.byref(ip), ctypes.byref(n))
    if rc != 0:
        raise ValueError("or_stem_items failed (k must be 3..31)")
    try:
        m = int(n.value)
        stems = np.ctypeslib.as_array(sp, shape=(max(m, 1),))[:m].copy()
        items = np.ctypeslib.as_array(ip, shape=(max(m, 1) * 32,))[:m * 32].copy()
    finally:
        lib.or_free_ptr(ctypes.cast(sp, ctypes.c_void_p))
        lib.or_free_ptr(ctypes.cast(ip, ctypes.c_void_p))
    return stems, items.reshape(m, 2, 16)


def filter_reads(k: int, n_counters: int, keys, counts, bases, offsets, tumour_min: int,
                 normal_max: int) -> np.ndarray:
    """Filter-unit lookup (kc_oracle.c, or_filter_reads; paper Sec. II-B):
    per read, the number of windows whose k-mer has tumour count >=
    tumour_min and normal count <= normal_max in the final table (keys
    ascending, counts [n, n_counters])."""
    lib = _load()
    keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
    counts = np.ascontiguousarray(counts, dtype=np.uint32).reshape(-1)
    bases, offsets, _ = _arrays(bases, offsets, None)
    n_reads = offsets.size - 1
    out = np.zeros(max(n_reads, 1), np.uint32)
    rc = lib.or_filter_reads(k, n_counters, _ptr(keys, U64P), _ptr(counts, U32P), keys.size,
                             _ptr(bases, U8P), _ptr(offsets, U64P), n_reads, tumour_min, normal_max,
                             _ptr(out, U32P))
    if rc != 0:
        raise ValueError("or_filter_reads failed")
    return out[:n_reads]


def sample_counts(params: Params, bases, offsets, sample_keys, tags=None, threads: int = 0):
    """Exact per-counter counts of distinct canonical keys (any order); also N_valid."""
    bases, offsets, tags = _arrays(bases, offsets, tags)
    keys = np.unique(np.asarray(sample_keys, dtype=np.uint64))
    out = np.zeros(max(keys.size * params.n_counters, 1), dtype=np.uint32)
    nv = ctypes.c_uint64(0)
    p = params.c()
    rc = _load().or_sample_counts(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P),
                                  offsets.size - 1, _ptr(tags, U8P), _ptr(keys, U64P), keys.size,
                                  _ptr(out, U32P), ctypes.byref(nv), threads or _threads())
    if rc:
        raise ValueError("or_sample_counts failed (%d)" % rc)
    return keys, out[:keys.size * params.n_counters].reshape(keys.size, params.n_counters), \
        int(nv.value)


def sample_hits(params: Params, bases, offsets, sample_bits, threads: int = 0):
    """min(2, hits(b)) for distinct bit positions (any order)."""
    bases, offsets, _ = _arrays(bases, offsets, None)
    bits = np.unique(np.asarray(sample_bits, dtype=np.uint64))
    out = np.zeros(max(bits.size, 1), dtype=np.uint32)
    p = params.c()
    rc = _load().or_sample_hits(ctypes.byref(p), _ptr(bases, U8P), _ptr(offsets, U64P),
                                offsets.size - 1, _ptr(bits, U64P), bits.size, _ptr(out, U32P),
                                threads or _threads())
    if rc:
        raise ValueError("or_sample_hits failed (%d)" % rc)
    return bits, out[:bits.size]


def _threads():
    return max(1, min(16, os.cpu_count() or 1))
