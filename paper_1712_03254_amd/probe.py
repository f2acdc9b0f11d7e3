"""Binding of libkc_probe.so, the LDS atomic throughput microbenchmark
(include/kc_probe.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB = os.path.join(HERE, "libkc_probe.so")
EXPORTED = ["kcp_lds_atomics"]
KCP_OR, KCP_OR_RTN, KCP_ADD = 0, 1, 2
THREADS = 1024

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(PROBE_LIB):
            raise RuntimeError("libkc_probe.so is not built (python -m paper_1712_03254_amd.build)")
        lib = ctypes.CDLL(PROBE_LIB)
        lib.kcp_lds_atomics.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_uint64)]
        lib.kcp_lds_atomics.restype = ctypes.c_int
        _lib = lib
    return _lib


def lds_atomics(kind: int, words_log2: int = 13, iters: int = 64, blocks: int = 4096):
    """Runs the microbenchmark once; returns (ops, ms, check) where ops is
    the number of atomics issued."""
    ms = ctypes.c_float(0.0)
    chk = ctypes.c_uint64(0)
    rc = load().kcp_lds_atomics(kind, words_log2, iters, blocks, ctypes.byref(ms), ctypes.byref(chk))
    if rc != 0:
        raise RuntimeError("kcp_lds_atomics failed (%d)" % rc)
    return blocks * THREADS * iters * 8, float(ms.value), int(chk.value)


def lds_atomic_peak(kind: int, words_log2: int = 13, reps: int = 3) -> float:
    """Best of `reps` runs (after one warm-up), in atomics per second."""
    lds_atomics(kind, words_log2, iters=8, blocks=512)
    best = 0.0
    for _ in range(reps):
        ops, ms, _ = lds_atomics(kind, words_log2)
        best = max(best, ops / (ms * 1e-3))
    return best
