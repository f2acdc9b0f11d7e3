"""Digests of whole outputs, for comparing results too large to store.

Test infrastructure: a serialisation and SHA-256 of arrays, holding none of
the counting arithmetic.  The committed digests under ``tests/golden/`` are
written from the CPU oracle's output by ``tests/golden/make_digests.py``; the
GPU tests digest the library's output the same way and compare.

Byte stream of a table: its entries in ascending key order, each the key as
a little-endian uint64 followed by its n_counters counts as little-endian
uint32.  The stream is also cut by value range (the top RANGE_BITS bits of
the 2k-bit code), so that a mismatch names the range it is in.  Bloom levels:
their little-endian uint64 words in order.
"""
from __future__ import annotations

import hashlib

import numpy as np

RANGE_BITS = 4


def table_bytes(keys_sorted: np.ndarray, counts_sorted: np.ndarray) -> np.ndarray:
    keys_sorted = np.asarray(keys_sorted, dtype=np.uint64).reshape(-1)
    counts_sorted = np.asarray(counts_sorted, dtype=np.uint32).reshape(keys_sorted.size, -1)
    nc = counts_sorted.shape[1]
    rec = np.empty(keys_sorted.size, dtype=np.dtype([("k", "<u8"), ("c", "<u4", (nc,))]))
    rec["k"] = keys_sorted
    rec["c"] = counts_sorted
    return rec


def table_digests(keys_sorted: np.ndarray, counts_sorted: np.ndarray, k: int) -> dict:
    """{'sha256': whole stream, 'ranges': [(entries, sum of counts, sha256)]}
    of a table already sorted by key."""
    keys_sorted = np.asarray(keys_sorted, dtype=np.uint64).reshape(-1)
    counts_sorted = np.asarray(counts_sorted, dtype=np.uint32).reshape(keys_sorted.size, -1)
    if keys_sorted.size > 1 and not bool(np.all(keys_sorted[1:] > keys_sorted[:-1])):
        raise ValueError("table keys are not strictly ascending")
    rb = min(RANGE_BITS, 2 * k)
    edges = np.searchsorted(keys_sorted, np.arange((1 << rb) + 1, dtype=np.uint64)
                            << np.uint64(2 * k - rb))
    whole = hashlib.sha256()
    ranges = []
    for q in range(1 << rb):
        lo, hi = int(edges[q]), int(edges[q + 1])
        blob = table_bytes(keys_sorted[lo:hi], counts_sorted[lo:hi]).tobytes()
        whole.update(blob)
        ranges.append((hi - lo, int(counts_sorted[lo:hi].sum(dtype=np.uint64)),
                       hashlib.sha256(blob).hexdigest()))
    return {"sha256": whole.hexdigest(), "ranges": ranges}


class TableDigest:
    """table_digests over a table handed over in ascending pieces (the
    oracle's value ranges, each wholly inside one digest range when the
    oracle uses at least RANGE_BITS range bits)."""

    def __init__(self, k: int):
        self.rb = min(RANGE_BITS, 2 * k)
        self.shift = 2 * k - self.rb
        self.whole = hashlib.sha256()
        self.parts = [[0, 0, hashlib.sha256()] for _ in range(1 << self.rb)]
        self.last = -1

    def update(self, keys_sorted: np.ndarray, counts_sorted: np.ndarray):
        keys_sorted = np.asarray(keys_sorted, dtype=np.uint64).reshape(-1)
        if keys_sorted.size == 0:
            return
        counts_sorted = np.asarray(counts_sorted, dtype=np.uint32).reshape(keys_sorted.size, -1)
        first = int(keys_sorted[0]) >> self.shift
        if int(keys_sorted[-1]) >> self.shift != first or first < self.last:
            raise ValueError("piece crosses a digest range or comes out of order")
        self.last = first
        blob = table_bytes(keys_sorted, counts_sorted).tobytes()
        self.whole.update(blob)
        part = self.parts[first]
        part[0] += keys_sorted.size
        part[1] += int(counts_sorted.sum(dtype=np.uint64))
        part[2].update(blob)

    def result(self) -> dict:
        return {"sha256": self.whole.hexdigest(),
                "ranges": [(n, s, h.hexdigest()) for n, s, h in self.parts]}


def words_digest(words: np.ndarray) -> str:
    # hashed in place (levels of 2^36 bits are 8 GiB each)
    return hashlib.sha256(memoryview(np.ascontiguousarray(words, dtype="<u8")).cast("B")).hexdigest()


STAT_KEYS = ["n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount",
             "b2_popcount"]


def write_digest_file(path: str, header: list[str], stats: dict, table: dict, b1: str, b2: str):
    with open(path, "w") as f:
        for line in header:
            f.write("# %s\n" % line)
        for name in STAT_KEYS:
            f.write("stat %s %d\n" % (name, stats[name]))
        f.write("table %s\n" % table["sha256"])
        for q, (n, s, h) in enumerate(table["ranges"]):
            f.write("range %d %d %d %s\n" % (q, n, s, h))
        f.write("b1 %s\n" % b1)
        f.write("b2 %s\n" % b2)


def read_digest_file(path: str) -> dict:
    out = {"stats": {}, "ranges": []}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "stat":
                out["stats"][parts[1]] = int(parts[2])
            elif parts[0] == "table":
                out["sha256"] = parts[1]
            elif parts[0] == "range":
                out["ranges"].append((int(parts[2]), int(parts[3]), parts[4]))
            elif parts[0] in ("b1", "b2"):
                out[parts[0]] = parts[1]
    return out


def served_subset(sizes, count: int = 16, seed: int = 0):
    """Indices (into the timed requests) of the served requests checked
    against the oracle: the largest and count - 1 others drawn with a seeded
    generator, ascending."""
    sizes = np.asarray(sizes)
    big = int(np.argmax(sizes))
    rest = np.array([i for i in range(sizes.size) if i != big])
    pick = np.random.default_rng(seed).choice(rest, size=min(count - 1, rest.size), replace=False)
    return sorted([big] + [int(i) for i in pick])


def write_request_digests(path: str, header: list[str], records: list[dict]):
    """One record per request: 'request i reads n normal s0 tumour s1 m M',
    then its statistics, table, ranges and levels, each line led by i."""
    with open(path, "w") as f:
        for line in header:
            f.write("# %s\n" % line)
        for r in records:
            i = r["index"]
            f.write("request %d reads %d normal %d tumour %d m %d\n" % (
                i, r["reads"], r["normal"], r["tumour"], r["m"]))
            for name in STAT_KEYS:
                f.write("stat %d %s %d\n" % (i, name, r["stats"][name]))
            f.write("table %d %s\n" % (i, r["table"]["sha256"]))
            for q, (n, s, h) in enumerate(r["table"]["ranges"]):
                f.write("range %d %d %d %d %s\n" % (i, q, n, s, h))
            f.write("b1 %d %s\n" % (i, r["b1"]))
            f.write("b2 %d %s\n" % (i, r["b2"]))


def read_request_digests(path: str) -> dict:
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            i = int(p[1])
            if p[0] == "request":
                out[i] = {"reads": int(p[3]), "normal": int(p[5]), "tumour": int(p[7]),
                          "m": int(p[9]), "stats": {}, "ranges": []}
            elif p[0] == "stat":
                out[i]["stats"][p[2]] = int(p[3])
            elif p[0] == "table":
                out[i]["sha256"] = p[2]
            elif p[0] == "range":
                out[i]["ranges"].append((int(p[3]), int(p[4]), p[5]))
            elif p[0] in ("b1", "b2"):
                out[i][p[0]] = p[2]
    return out
