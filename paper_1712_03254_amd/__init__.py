"""Python binding of libkc.so, the MI355X k-mer counter (C ABI in include/kc.h).

Argument marshalling only: every step of the counting path runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  Importing
this module does not need a GPU; creating a counter does, and a missing or
unloadable library raises instead of falling back to anything.

The functions mirror the C entry points one to one (``kc_create``,
``kc_insert_reads``, ``kc_finalize``, ``kc_query``, ``kc_spill``,
``kc_export``, ...).  ``KmerCounter`` wraps them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkc.so")
_lib = None

KC_OK = 0
KC_ERR_INVALID_ARG = -1
KC_ERR_OUT_OF_MEMORY = -2
KC_ERR_BAD_STATE = -3
KC_ERR_DEVICE = -4
KC_ERR_OVER_BUDGET = -5

STAGES = ["pack", "level1", "scan", "level2", "bloom", "tally", "unify", "query", "spill", "graph",
          "stems", "filter"]

EXPORTED = ["kc_abi_version", "kc_status_str", "kc_create", "kc_insert_reads", "kc_finalize",
            "kc_query", "kc_spill", "kc_export", "kc_export_bloom", "kc_export_bloom_words",
            "kc_debug_keys",
            "kc_get_stats", "kc_reset", "kc_destroy", "kc_last_error", "kc_count_batch",
            "kc_autotune_batch", "kc_server_create", "kc_server_submit", "kc_server_wait",
            "kc_server_release", "kc_server_usage", "kc_server_destroy", "kc_server_set_overlap",
            "kc_server_plan_admission",
            "kc_export_stems", "kc_filter_reads", "kc_filter_reads_noalloc", "kc_checkpoint",
            "kc_restore"]


class KcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


class KcConfig(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("n_counters", ctypes.c_uint32),
                ("min_count", ctypes.c_uint32), ("bloom_bits_log2", ctypes.c_uint32),
                ("bloom_hashes", ctypes.c_uint32), ("bloom_block_log2", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("partitions_log2", ctypes.c_uint32),
                ("table_slots", ctypes.c_uint32), ("scatter_bits", ctypes.c_uint32),
                ("group_bases_log2", ctypes.c_uint32),
                ("hbm_table_budget_bytes", ctypes.c_uint64),
                ("shuffle_tile_log2", ctypes.c_uint32), ("reserved_", ctypes.c_uint32)]


class KcStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount",
        "b2_popcount", "spilled_partitions", "spilled_bytes", "overflow_keys",
        "passed_distinct")] + [
        ("partitions_log2", ctypes.c_uint32), ("table_slots", ctypes.c_uint32),
        ("n_segments", ctypes.c_uint32), ("retries", ctypes.c_uint32),
        ("kernel_ms", ctypes.c_double * 16), ("kernel_launches", ctypes.c_uint64 * 16)]

    def as_dict(self) -> dict:
        d = {n: getattr(self, n) for n, _ in self._fields_[:15]}
        d["kernel_ms"] = {STAGES[i]: self.kernel_ms[i] for i in range(len(STAGES))}
        d["kernel_launches"] = {STAGES[i]: int(self.kernel_launches[i]) for i in range(len(STAGES))}
        return d


class KcChunk(ctypes.Structure):
    _fields_ = [("bases_dev", ctypes.c_void_p), ("offsets_dev", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint64), ("total_bases", ctypes.c_uint64)]


class KcRequest(ctypes.Structure):
    _fields_ = [("cfg", KcConfig), ("parts", KcChunk * 2), ("n_parts", ctypes.c_uint32),
                ("reserved_", ctypes.c_uint32), ("ready_event", ctypes.c_void_p)]


class KcResponse(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("worker", ctypes.c_uint32), ("stats", KcStats),
                ("ctx", ctypes.c_void_p), ("submit_ms", ctypes.c_double),
                ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("footprint_bytes", ctypes.c_uint64)]


class KcServerStats(ctypes.Structure):
    _fields_ = [("in_use_bytes", ctypes.c_uint64), ("pooled_bytes", ctypes.c_uint64),
                ("queued", ctypes.c_uint32), ("running", ctypes.c_uint32),
                ("pooled_contexts", ctypes.c_uint32), ("reserved_", ctypes.c_uint32),
                ("created", ctypes.c_uint64), ("reused", ctypes.c_uint64),
                ("grown", ctypes.c_uint64), ("evicted", ctypes.c_uint64),
                ("cached_bytes", ctypes.c_uint64), ("device_allocs", ctypes.c_uint64),
                ("device_frees", ctypes.c_uint64)]


class KcAdmitPooled(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64), ("after", ctypes.c_uint64), ("stamp", ctypes.c_uint64)]


class KcAdmitState(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_uint64), ("in_use", ctypes.c_uint64),
                ("pooled", ctypes.c_uint64), ("max_inflight", ctypes.c_uint64),
                ("inflight", ctypes.c_uint64), ("running", ctypes.c_uint32),
                ("reserved_", ctypes.c_uint32)]


class KcTuneTrial(ctypes.Structure):
    _fields_ = [("partitions_log2", ctypes.c_uint32), ("table_slots", ctypes.c_uint32),
                ("scatter_bits", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("ms", ctypes.c_double), ("overflow_keys", ctypes.c_uint64),
                ("shuffle_tile_log2", ctypes.c_uint32), ("reserved_", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_ if n != "reserved_"}


def _status_name(s: int) -> str:
    return {0: "KC_OK", -1: "KC_ERR_INVALID_ARG", -2: "KC_ERR_OUT_OF_MEMORY",
            -3: "KC_ERR_BAD_STATE", -4: "KC_ERR_DEVICE", -5: "KC_ERR_OVER_BUDGET"}.get(s, str(s))


def load():
    """Loads libkc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libkc.so is not built (run __graft_entry__.build() or "
                          "python paper_1712_03254_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    V, P, U32, U64, I64 = ctypes.c_void_p, ctypes.POINTER, ctypes.c_uint32, ctypes.c_uint64, \
        ctypes.c_int64
    st = ctypes.c_int
    sig = {
        "kc_abi_version": ([], U32),
        "kc_status_str": ([st], ctypes.c_char_p),
        "kc_create": ([P(KcConfig), ctypes.c_int, P(V)], st),
        "kc_insert_reads": ([V, V, V, U64, U64, U32, V], st),
        "kc_finalize": ([V, V, P(KcStats)], st),
        "kc_query": ([V, V, U64, V, V], st),
        "kc_spill": ([V, I64, P(U64)], st),
        "kc_export": ([V, V, V, U64, P(U64)], st),
        "kc_export_bloom": ([V, V, V, U64], st),
        "kc_export_bloom_words": ([V, V, U64, V, V], st),
        "kc_export_stems": ([V, V, V, U64, P(U64), V], st),
        "kc_filter_reads": ([V, V, V, U64, U64, U32, U32, V, V], st),
        "kc_filter_reads_noalloc": ([V, V, V, U64, U64, U32, U32, V, V], st),
        "kc_checkpoint": ([V, ctypes.c_char_p], st),
        "kc_restore": ([ctypes.c_char_p, ctypes.c_int, P(V)], st),
        "kc_debug_keys": ([V, V, V, U64, P(U64)], st),
        "kc_get_stats": ([V, P(KcStats)], st),
        "kc_reset": ([V], st),
        "kc_destroy": ([V], None),
        "kc_last_error": ([V], ctypes.c_char_p),
        "kc_count_batch": ([V, P(KcChunk), U32, U32, V, P(KcStats)], st),
        "kc_autotune_batch": ([P(KcConfig), ctypes.c_int, P(KcChunk), U32, U32, V, P(KcConfig),
                               P(KcTuneTrial), U32, P(U32)], st),
        "kc_server_create": ([ctypes.c_int, U64, U32, P(V)], st),
        "kc_server_submit": ([V, P(KcRequest), P(U64)], st),
        "kc_server_wait": ([V, U64, P(KcResponse)], st),
        "kc_server_release": ([V, U64], st),
        "kc_server_usage": ([V, P(KcServerStats)], st),
        "kc_server_destroy": ([V], None),
        "kc_server_set_overlap": ([V, U64], st),
        "kc_server_plan_admission": ([P(KcAdmitState), P(KcAdmitPooled), U32, U64, U64, P(U32),
                                      P(ctypes.c_int32), P(U64), P(U32), P(U32)], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(ctx, status: int):
    if status != KC_OK:
        msg = load().kc_last_error(ctx)
        raise KcError(status, msg.decode() if msg else "")


# ---- one-to-one wrappers of the C entry points ------------------------------

def kc_abi_version() -> int:
    return int(load().kc_abi_version())


def kc_create(cfg: KcConfig, device: int = 0):
    h = ctypes.c_void_p()
    _check(None, load().kc_create(ctypes.byref(cfg), device, ctypes.byref(h)))
    return h


def kc_checkpoint(ctx, path: str):
    _check(ctx, load().kc_checkpoint(ctx, os.fsencode(path)))


def kc_restore(path: str, device: int = 0):
    h = ctypes.c_void_p()
    _check(None, load().kc_restore(os.fsencode(path), device, ctypes.byref(h)))
    return h


def checkpoint_config(path: str) -> "Config":
    """The configuration stored in a checkpoint's header (it follows an
    8-byte magic, the ABI version, a reserved word and the header size)."""
    with open(path, "rb") as f:
        raw = f.read(24 + ctypes.sizeof(KcConfig))
    if len(raw) < 24 + ctypes.sizeof(KcConfig):
        raise ValueError("%s is too short to be a checkpoint" % path)
    return Config.from_c(KcConfig.from_buffer_copy(raw, 24))


def kc_insert_reads(ctx, bases_ptr: int, offsets_ptr: int, n_reads: int, total_bases: int,
                    counter: int, stream_ptr: int):
    _check(ctx, load().kc_insert_reads(ctx, bases_ptr, offsets_ptr, n_reads, total_bases,
                                       counter, stream_ptr))


def kc_finalize(ctx, stream_ptr: int) -> KcStats:
    s = KcStats()
    _check(ctx, load().kc_finalize(ctx, stream_ptr, ctypes.byref(s)))
    return s


def kc_query(ctx, kmers_ptr: int, n: int, counts_ptr: int, stream_ptr: int):
    _check(ctx, load().kc_query(ctx, kmers_ptr, n, counts_ptr, stream_ptr))


def kc_spill(ctx, partition: int = -1) -> int:
    b = ctypes.c_uint64(0)
    _check(ctx, load().kc_spill(ctx, partition, ctypes.byref(b)))
    return int(b.value)


def kc_export(ctx, n_counters: int):
    n = ctypes.c_uint64(0)
    lib = load()
    _check(ctx, lib.kc_export(ctx, None, None, 0, ctypes.byref(n)))
    e = int(n.value)
    keys = np.empty(max(e, 1), dtype=np.uint64)
    counts = np.empty(max(e * n_counters, 1), dtype=np.uint32)
    _check(ctx, lib.kc_export(ctx, keys.ctypes.data, counts.ctypes.data, e, ctypes.byref(n)))
    return keys[:e], counts[:e * n_counters].reshape(e, n_counters)


def kc_export_stems(ctx, stems_ptr: int, counts_ptr: int, capacity: int, stream: int = 0) -> int:
    """Writes the stem items into device buffers; returns their number."""
    n = ctypes.c_uint64(0)
    _check(ctx, load().kc_export_stems(ctx, stems_ptr, counts_ptr, capacity, ctypes.byref(n), stream))
    return int(n.value)


def kc_export_bloom(ctx, words: int):
    b1 = np.empty(words, dtype=np.uint64)
    b2 = np.empty(words, dtype=np.uint64)
    _check(ctx, load().kc_export_bloom(ctx, b1.ctypes.data, b2.ctypes.data, words))
    return b1, b2


def kc_export_bloom_words(ctx, word_idx):
    idx = np.ascontiguousarray(word_idx, dtype=np.uint64)
    b1 = np.empty(max(idx.size, 1), dtype=np.uint64)
    b2 = np.empty(max(idx.size, 1), dtype=np.uint64)
    _check(ctx, load().kc_export_bloom_words(ctx, idx.ctypes.data, idx.size, b1.ctypes.data,
                                             b2.ctypes.data))
    return b1[:idx.size], b2[:idx.size]


def kc_debug_keys(ctx):
    n = ctypes.c_uint64(0)
    lib = load()
    _check(ctx, lib.kc_debug_keys(ctx, None, None, 0, ctypes.byref(n)))
    e = int(n.value)
    keys = np.empty(max(e, 1), dtype=np.uint64)
    part = np.empty(max(e, 1), dtype=np.uint32)
    _check(ctx, lib.kc_debug_keys(ctx, keys.ctypes.data, part.ctypes.data, e, ctypes.byref(n)))
    return keys[:e], part[:e]


def _chunk_array(chunks):
    arr = (KcChunk * max(1, len(chunks)))()
    for i, (b, o, n, t) in enumerate(chunks):
        arr[i] = KcChunk(b, o, n, t)
    return arr


def kc_count_batch(ctx, chunks, counter: int, stream_ptr: int) -> KcStats:
    """chunks: list of (bases_ptr, offsets_ptr, n_reads, total_bases)."""
    s = KcStats()
    arr = _chunk_array(chunks)
    _check(ctx, load().kc_count_batch(ctx, arr, len(chunks), counter, stream_ptr, ctypes.byref(s)))
    return s


def kc_autotune_batch(cfg: KcConfig, device: int, chunks, counter: int, stream_ptr: int):
    """Returns (best KcConfig, list of trial dicts)."""
    arr = _chunk_array(chunks)
    best = KcConfig()
    trials = (KcTuneTrial * 64)()
    n = ctypes.c_uint32(0)
    _check(None, load().kc_autotune_batch(ctypes.byref(cfg), device, arr, len(chunks), counter,
                                          stream_ptr, ctypes.byref(best), trials, 64,
                                          ctypes.byref(n)))
    return best, [trials[i].as_dict() for i in range(min(n.value, 64))]


def kc_get_stats(ctx) -> KcStats:
    s = KcStats()
    _check(ctx, load().kc_get_stats(ctx, ctypes.byref(s)))
    return s


def kc_reset(ctx):
    _check(ctx, load().kc_reset(ctx))


def kc_destroy(ctx):
    if ctx:
        load().kc_destroy(ctx)


def kc_last_error(ctx=None) -> str:
    m = load().kc_last_error(ctx)
    return m.decode() if m else ""


# ---- convenience wrapper ------------------------------------------------------

@dataclass
class Config:
    k: int = 31
    n_counters: int = 1
    min_count: int = 2
    bloom_bits_log2: int = 24
    bloom_hashes: int = 3
    bloom_block_log2: int = 19
    seed: int = 0
    partitions_log2: int = 0
    table_slots: int = 0
    scatter_bits: int = 0
    hbm_table_budget_bytes: int = 0
    group_bases_log2: int = 0
    shuffle_tile_log2: int = 0

    def c(self) -> KcConfig:
        return KcConfig(self.k, self.n_counters, self.min_count, self.bloom_bits_log2,
                        self.bloom_hashes, min(self.bloom_block_log2, self.bloom_bits_log2),
                        self.seed & ((1 << 64) - 1), self.partitions_log2, self.table_slots,
                        self.scatter_bits, self.group_bases_log2, self.hbm_table_budget_bytes,
                        self.shuffle_tile_log2, 0)

    @staticmethod
    def from_c(c: KcConfig) -> "Config":
        return Config(c.k, c.n_counters, c.min_count, c.bloom_bits_log2, c.bloom_hashes,
                      c.bloom_block_log2, c.seed, c.partitions_log2, c.table_slots,
                      c.scatter_bits, c.hbm_table_budget_bytes, c.group_bases_log2,
                      c.shuffle_tile_log2)


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def chunk_list(chunks):
    """(bases, offsets) device tensor pairs -> kc_chunk tuples."""
    out = []
    for b, o in chunks:
        out.append((b.data_ptr() if b.numel() else 0, o.data_ptr(), o.numel() - 1, b.numel()))
    return out


def autotune_batch(cfg: Config, chunks, counter: int = 0, device: int = 0, stream=None):
    """Measured choice of partitions, table slots and shuffle split for a batch
    (kc_autotune_batch).  Returns (best Config, trial records)."""
    best, trials = kc_autotune_batch(cfg.c(), device, chunk_list(chunks), counter,
                                     _stream_ptr(stream))
    return Config.from_c(best), trials


class KmerCounter:
    """One counting context on one GPU; inputs and outputs are torch tensors."""

    def __init__(self, cfg: Config, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("KmerCounter needs a HIP device")
        self.cfg = cfg
        self.device = device
        self.ctx = kc_create(cfg.c(), device)

    def close(self):
        if self.ctx:
            kc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def checkpoint(self, path: str):
        """Writes the finalized context to `path` (kc_checkpoint)."""
        kc_checkpoint(self.ctx, path)

    @classmethod
    def restore(cls, path: str, device: int = 0) -> "KmerCounter":
        """A finalized counter read back from a checkpoint (kc_restore)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("KmerCounter needs a HIP device")
        obj = cls.__new__(cls)
        obj.cfg = checkpoint_config(path)
        obj.device = device
        obj.ctx = kc_restore(path, device)
        return obj

    def insert_reads(self, bases, offsets, counter: int = 0, stream=None):
        """bases: uint8 device tensor; offsets: int64/uint64 device tensor of n_reads+1."""
        n_reads = offsets.numel() - 1
        kc_insert_reads(self.ctx, bases.data_ptr() if bases.numel() else 0, offsets.data_ptr(),
                        n_reads, bases.numel(), counter, _stream_ptr(stream))

    def finalize(self, stream=None) -> dict:
        return kc_finalize(self.ctx, _stream_ptr(stream)).as_dict()

    def query(self, kmers, stream=None):
        import torch
        out = torch.empty((kmers.numel(), self.cfg.n_counters), dtype=torch.int32,
                          device=kmers.device)
        kc_query(self.ctx, kmers.data_ptr(), kmers.numel(), out.data_ptr(), _stream_ptr(stream))
        return out

    def count_batch(self, chunks, counter: int = 0, stream=None) -> dict:
        """chunks: list of (bases, offsets) device tensor pairs; inserts them all
        and finalizes, as one graph launch (kc_count_batch)."""
        return kc_count_batch(self.ctx, chunk_list(chunks), counter, _stream_ptr(stream)).as_dict()

    def spill(self, partition: int = -1) -> int:
        return kc_spill(self.ctx, partition)

    def export(self):
        return kc_export(self.ctx, self.cfg.n_counters)

    def export_bloom(self):
        words = max(1, (1 << self.cfg.bloom_bits_log2) // 64)
        return kc_export_bloom(self.ctx, words)

    def export_bloom_words(self, word_idx):
        """Words word_idx (uint64 indices) of both Bloom levels (kc_export_bloom_words)."""
        return kc_export_bloom_words(self.ctx, word_idx)

    def filter_reads(self, bases, offsets, tumour_min: int, normal_max: int, stream=None):
        """Filter-unit lookup (kc_filter_reads): per read of the batch, its
        windows whose k-mer has tumour count >= tumour_min and normal count
        <= normal_max.  bases uint8 / offsets int64 device tensors; returns an
        int32 device tensor (counts, read as unsigned)."""
        import torch
        n = offsets.numel() - 1
        out = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
        _check(self.ctx, load().kc_filter_reads(self.ctx, bases.data_ptr(), offsets.data_ptr(), n,
                                                 bases.numel(), tumour_min, normal_max,
                                                 out.data_ptr(), _stream_ptr(stream)))
        return out[:n]

    def filter_reads_noalloc(self, bases, offsets, tumour_min: int, normal_max: int, out,
                             stream=None):
        """kc_filter_reads_noalloc: as filter_reads, into the caller's int32
        device tensor `out` (n_reads entries), with no allocation inside."""
        n = offsets.numel() - 1
        _check(self.ctx, load().kc_filter_reads_noalloc(
            self.ctx, bases.data_ptr(), offsets.data_ptr(), n, bases.numel(), tumour_min,
            normal_max, out.data_ptr(), _stream_ptr(stream)))
        return out[:n]

    def export_stems(self, stream=None):
        """Stem items of the final table (kc_export_stems), as device tensors:
        stems int64[n] (codes of k-2 bases) and counts int16[n, 2, 16]
        (counter, 4a+b), 16-bit counts read as unsigned."""
        import torch
        cap = max(1, self.stats()["entries"])
        stems = torch.empty(cap, dtype=torch.int64, device="cuda")
        counts = torch.empty((cap, 2, 16), dtype=torch.int16, device="cuda")
        n = kc_export_stems(self.ctx, stems.data_ptr(), counts.data_ptr(), cap, _stream_ptr(stream))
        return stems[:n], counts[:n]

    def debug_keys(self):
        return kc_debug_keys(self.ctx)

    def stats(self) -> dict:
        return kc_get_stats(self.ctx).as_dict()

    def reset(self):
        kc_reset(self.ctx)


# ---- served form ----------------------------------------------------------------

class Server:
    """Request server (kc_server_*): jobs of their own configuration, admitted
    under an HBM budget, run concurrently by `workers` threads.  With
    overlap_bases > 0, a request starts only when none runs or the running
    ones and it hold at most that many bases (kc_server_set_overlap)."""

    def __init__(self, budget_bytes: int, workers: int = 4, device: int = 0,
                 overlap_bases: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Server needs a HIP device")
        h = ctypes.c_void_p()
        _check(None, load().kc_server_create(device, budget_bytes, workers, ctypes.byref(h)))
        self.h = h
        self._held = {}  # ticket -> (event, part tensors) until the request is done
        if overlap_bases:
            self.set_overlap(overlap_bases)

    def set_overlap(self, max_inflight_bases: int):
        _check(None, load().kc_server_set_overlap(self.h, max_inflight_bases))

    def submit(self, cfg: Config, parts) -> int:
        """parts: list of up to two (bases, offsets) device tensor pairs (part c
        counted into counter c).  Returns the ticket at once.  The worker waits
        for the work queued so far on the current stream (which may still be
        writing the reads), and the tensors are held until the request is done."""
        import torch
        r = KcRequest()
        r.cfg = cfg.c()
        for i, (b, o, n, t) in enumerate(chunk_list(parts)):
            r.parts[i] = KcChunk(b, o, n, t)
        r.n_parts = len(parts)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        r.ready_event = ev.cuda_event
        t = ctypes.c_uint64(0)
        _check(None, load().kc_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        self._held[int(t.value)] = (ev, list(parts))
        return int(t.value)

    def wait(self, ticket: int) -> KcResponse:
        out = KcResponse()
        _check(None, load().kc_server_wait(self.h, ticket, ctypes.byref(out)))
        self._held.pop(ticket, None)
        return out

    def release(self, ticket: int):
        _check(None, load().kc_server_release(self.h, ticket))
        self._held.pop(ticket, None)

    def usage(self) -> dict:
        st = KcServerStats()
        _check(None, load().kc_server_usage(self.h, ctypes.byref(st)))
        d = {n: getattr(st, n) for n, _ in st._fields_ if n != "reserved_"}
        d["in_use"], d["pooled"] = d["in_use_bytes"], d["pooled_bytes"]
        return d

    def close(self):
        if self.h:
            load().kc_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_admission(budget: int, in_use: int, pool, job_bases: int, estimate: int,
                   max_inflight: int = 0, inflight: int = 0, running: int = 0):
    """kc_server_plan_admission on plain numbers (no device needed).  pool:
    list of (bytes now, bytes after the job or 0, last-use stamp).  Returns
    None when the request must wait, else (choice: pooled index or -1 for a
    new context, reserved bytes, pooled indices to evict in order)."""
    n = len(pool)
    arr = (KcAdmitPooled * max(1, n))()
    for i, (b, a, s) in enumerate(pool):
        arr[i] = KcAdmitPooled(b, a, s)
    state = KcAdmitState(budget, in_use, sum(p[0] for p in pool), max_inflight, inflight, running,
                         0)
    admit, nev = ctypes.c_uint32(0), ctypes.c_uint32(0)
    choice, reserve = ctypes.c_int32(0), ctypes.c_uint64(0)
    ev = (ctypes.c_uint32 * max(1, n))()
    _check(None, load().kc_server_plan_admission(ctypes.byref(state), arr, n, job_bases, estimate,
                                                 ctypes.byref(admit), ctypes.byref(choice),
                                                 ctypes.byref(reserve), ev, ctypes.byref(nev)))
    if not admit.value:
        return None
    return int(choice.value), int(reserve.value), [int(ev[i]) for i in range(nev.value)]


def response_table(resp: KcResponse, n_counters: int):
    """(keys, counts) of a finished request, from its resident context."""
    return kc_export(ctypes.c_void_p(resp.ctx), n_counters)


def response_query(resp: KcResponse, kmers, n_counters: int):
    import torch
    out = torch.empty((kmers.numel(), n_counters), dtype=torch.int32, device=kmers.device)
    kc_query(ctypes.c_void_p(resp.ctx), kmers.data_ptr(), kmers.numel(), out.data_ptr(),
             _stream_ptr(None))
    return out
