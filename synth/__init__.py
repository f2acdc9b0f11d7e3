"""Seeded synthetic genomes and reads (input generation only).

The C source ``synth.c`` holds the generator; this module builds it with gcc
(``build()``), loads it with ctypes and returns numpy arrays.  Nothing here
encodes, hashes or counts k-mers: the counting method lives elsewhere, and both
the CPU oracle and the GPU library read what these functions return.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

U64P = ctypes.POINTER(ctypes.c_uint64)
U8P = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so (gcc, -O2, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.synth_genome.argtypes = [ctypes.c_uint64, ctypes.c_uint64, U8P, ctypes.c_int]
        lib.synth_tumour.argtypes = [ctypes.c_uint64, U8P, ctypes.c_uint64, U8P, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_read_offsets.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint32, U64P]
        lib.synth_reads.argtypes = [ctypes.c_uint64, U8P, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_double, ctypes.c_double, U64P, U8P, ctypes.c_int]
        lib.synth_chunk_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_double, U64P]
        lib.synth_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, U64P]
        for f in (lib.synth_genome, lib.synth_tumour, lib.synth_read_offsets, lib.synth_reads,
                  lib.synth_chunk_sizes, lib.synth_draws):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads(threads):
    if threads:
        return int(threads)
    return max(1, min(16, os.cpu_count() or 1))


def _p8(a):
    return a.ctypes.data_as(U8P)


def _p64(a):
    return a.ctypes.data_as(U64P)


def genome(seed: int, length: int, threads: int = 0) -> np.ndarray:
    """Uniform i.i.d. ACGT genome of ``length`` bases (uint8 ASCII)."""
    out = np.empty(int(length), dtype=np.uint8)
    rc = _load().synth_genome(seed, length, _p8(out), _threads(threads))
    if rc:
        raise ValueError("synth_genome failed (%d)" % rc)
    return out


def tumour(seed: int, normal: np.ndarray, n_snv: int, n_inv: int, inv_min: int,
           inv_max: int) -> np.ndarray:
    """Normal genome plus distinct point substitutions, then in-place inversions."""
    normal = np.ascontiguousarray(normal, dtype=np.uint8)
    out = np.empty_like(normal)
    rc = _load().synth_tumour(seed, _p8(normal), normal.size, _p8(out), n_snv, n_inv, inv_min,
                              inv_max)
    if rc:
        raise ValueError("synth_tumour failed (%d)" % rc)
    return out


def read_offsets(seed: int, first: int, n: int, lmin: int, lmax: int) -> np.ndarray:
    off = np.empty(int(n) + 1, dtype=np.uint64)
    rc = _load().synth_read_offsets(seed, first, n, lmin, lmax, _p64(off))
    if rc:
        raise ValueError("synth_read_offsets failed (%d)" % rc)
    return off


def reads(seed: int, genome_seq: np.ndarray, first: int, n: int, lmin: int, lmax: int,
          err: float, nrate: float = 0.0, threads: int = 0):
    """Reads ``first .. first+n-1``: returns (bases uint8[total], offsets uint64[n+1])."""
    genome_seq = np.ascontiguousarray(genome_seq, dtype=np.uint8)
    off = read_offsets(seed, first, n, lmin, lmax)
    bases = np.empty(int(off[-1]), dtype=np.uint8)
    rc = _load().synth_reads(seed, _p8(genome_seq), genome_seq.size, first, n, lmin, lmax,
                             float(err), float(nrate), _p64(off), _p8(bases), _threads(threads))
    if rc:
        raise ValueError("synth_reads failed (%d)" % rc)
    return bases, off


def chunk_sizes(seed: int, n_chunks: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(int(n_chunks), dtype=np.uint64)
    rc = _load().synth_chunk_sizes(seed, n_chunks, float(lo), float(hi), _p64(out))
    if rc:
        raise ValueError("synth_chunk_sizes failed (%d)" % rc)
    return out


def draws(seed: int, stream_id: int, n: int) -> np.ndarray:
    out = np.empty(int(n), dtype=np.uint64)
    _load().synth_draws(seed, stream_id, n, _p64(out))
    return out


@dataclass(frozen=True)
class Workload:
    """A synthetic workload and the counting parameters it is run with."""
    name: str
    seed: int
    genome_len: int
    n_reads: int
    lmin: int
    lmax: int
    err: float
    nrate: float
    k: int
    bloom_bits_log2: int
    bloom_hashes: int
    bloom_block_log2: int
    partitions_log2: int
    n_counters: int = 1
    min_count: int = 2
    table_budget: int = 0
    batch_chunks: int = 0     # batched workloads: number of read chunks
    chunk_lo: float = 0.0     # reads per chunk, log-uniform in [chunk_lo, chunk_hi]
    chunk_hi: float = 0.0
    requests: int = 0         # served workloads: timed requests (after warm-up ones)
    warmup_requests: int = 0
    req_lo: float = 0.0       # reads per request, log-uniform in [req_lo, req_hi]
    req_hi: float = 0.0
    snv_rate: float = 0.0     # tumour genome: distinct point substitutions per base
    n_inv: int = 0            # ... then this many inversions of inv_lo..inv_hi bases
    inv_lo: int = 0
    inv_hi: int = 0
    serve_budget: int = 0     # HBM budget of the request server (bytes)

    def make_genome(self, threads: int = 0) -> np.ndarray:
        return genome(self.seed, self.genome_len, threads)

    def make_reads(self, genome_seq, first: int = 0, n: int | None = None, threads: int = 0):
        n = self.n_reads - first if n is None else n
        return reads(self.seed, genome_seq, first, n, self.lmin, self.lmax, self.err, self.nrate,
                     threads)

    def make_tumour(self, normal_seq) -> np.ndarray:
        return tumour(self.seed, normal_seq, int(self.snv_rate * self.genome_len), self.n_inv,
                      self.inv_lo, self.inv_hi)

    def make_sample_reads(self, genome_seq, sample: int, threads: int = 0):
        """Reads of sample 0 (normal) or 1 (tumour): disjoint index ranges of
        one read stream, so the two samples draw independent reads."""
        return self.make_reads(genome_seq, first=sample * self.n_reads, n=self.n_reads,
                               threads=threads)

    def request_plan(self):
        """(reads, normal start, tumour start) per request, warm-up ones first:
        size log-uniform in [req_lo, req_hi] (even), half from each sample, at
        seeded starts."""
        n = self.warmup_requests + self.requests
        d = draws(self.seed, 1, 3 * n).reshape(n, 3)
        u = (d[:, 0] >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        size = np.floor(np.exp(np.log(self.req_lo) + u * (np.log(self.req_hi) -
                                                           np.log(self.req_lo)))).astype(np.int64)
        half = np.maximum(1, size // 2)
        room = (self.n_reads - half + 1).astype(np.uint64)
        s0 = (d[:, 1] % room).astype(np.int64)
        s1 = (d[:, 2] % room).astype(np.int64)
        return np.stack([2 * half, s0, s1], axis=1)

    def request_params(self, n_reads: int):
        """Counting parameters of a served request of n_reads fixed-length
        reads: (k-mer windows, Bloom bits log2, partitions log2).  The Bloom
        filter has 2^m bits, m = clamp(ceil(log2(8 * windows)), 20, 34); the
        partition count (result-neutral) is about one per 2^13 bases, and at
        least one per Bloom block."""
        kmers = int(n_reads) * max(0, self.lmax - self.k + 1)
        m = int(min(34, max(20, math.ceil(math.log2(max(1, 8 * kmers))))))
        pl = max(m - self.bloom_block_log2,
                 int(round(math.log2(max(1, int(n_reads) * self.lmax) / 8192))))
        return kmers, m, pl

    def chunk_plan(self) -> np.ndarray:
        """Reads per chunk of a batched workload: floor(exp(U[ln lo, ln hi])),
        seeded; the chunks hold consecutive reads of one read stream."""
        return chunk_sizes(self.seed, self.batch_chunks, self.chunk_lo, self.chunk_hi)

    def make_chunk(self, genome_seq, sizes: np.ndarray, i: int, threads: int = 0):
        first = int(sizes[:i].sum())
        return self.make_reads(genome_seq, first=first, n=int(sizes[i]), threads=threads)


# The five workloads.  Partition counts are result-neutral; the value here is
# the one the GPU path runs with (each partition's table lives in LDS, so the
# count is set from the expected distinct k-mers per Bloom block).  Bloom
# blocks are 2^16 bits where the partitions allow it: a Bloom workgroup takes
# four such blocks (64 KiB of LDS for both levels, two workgroups per CU), and
# the count kernel screens against an 8 KiB level that stays in the CU's cache.
# The batched workload keeps 2^18-bit blocks: at 2^35 bits, 2^16-bit blocks
# would force 2^19 partitions, past the autotuner's choice.
WORKLOADS = {
    "plain_1mbp": Workload("plain_1mbp", 1, 1_000_000, 20_000, 100, 100, 0.01, 0.0,
                           31, 24, 3, 16, 8),
    "plain_100mbp": Workload("plain_100mbp", 2, 100_000_000, 10_000_000, 100, 100, 0.005, 0.001,
                             31, 32, 4, 16, 16),
    "batched_200mbp": Workload("batched_200mbp", 3, 200_000_000, 0, 100, 250, 0.005, 0.0,
                               31, 35, 4, 18, 19, batch_chunks=256, chunk_lo=1e3, chunk_hi=2e6),
    "served_300mbp": Workload("served_300mbp", 4, 300_000_000, 30_000_000, 100, 100, 0.005, 0.0,
                              31, 32, 4, 16, 16, n_counters=2, requests=512, warmup_requests=32,
                              req_lo=1e4, req_hi=5e6, snv_rate=0.001, n_inv=200, inv_lo=1000,
                              inv_hi=10000, serve_budget=32 << 30),
    "spill_3gbp": Workload("spill_3gbp", 5, 3_000_000_000, 200_000_000, 100, 100, 0.01, 0.0,
                           31, 36, 4, 16, 20, table_budget=64 << 30),
}
