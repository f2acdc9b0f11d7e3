"""Pins of the oracle's Filter-unit lookup (paper Sec. II-B: the input is
read again and its k-mers looked up in the frequency table to select
imbalanced ones): a hand-worked example, a string-level brute force and the
invariant that with no threshold every window whose k-mer is in the table is
selected."""
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "filter_example.txt")


def _pack(reads):
    bases = np.frombuffer("".join(reads).encode(), np.uint8) if reads else np.zeros(0, np.uint8)
    offs = np.concatenate([[0], np.cumsum([len(r) for r in reads])]).astype(np.uint64)
    return bases, offs


def test_filter_worked_example():
    f = {"table": [], "read": []}
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key in f:
            f[key].append(vals)
        else:
            f[key] = int(vals[0])
    table = sorted((brute.encode(s), int(n), int(t)) for s, n, t in f["table"])
    keys = np.array([x for x, _, _ in table], np.uint64)
    counts = np.array([[n, t] for _, n, t in table], np.uint32)
    reads = [r for r, _ in f["read"]]
    want = [int(v) for _, v in f["read"]]
    b, o = _pack(reads)
    got = oracle.filter_reads(f["k"], 2, keys, counts, b, o, f["tumour_min"], f["normal_max"])
    assert got.tolist() == want
    d = {x: (n, t) for x, n, t in table}
    assert brute.filter_reads(d, reads, f["k"], f["tumour_min"], f["normal_max"]) == want


@pytest.mark.parametrize("k,nc,tmin,nmax", [(3, 2, 1, 0), (5, 2, 2, 1), (9, 2, 3, 100), (9, 1, 2, 0),
                                            (21, 2, 1, 5)])
def test_filter_matches_brute_force(k, nc, tmin, nmax):
    rng = np.random.default_rng(k * 10 + nc)
    genome = "".join(rng.choice(list("ACGT"), 600))
    reads = []
    for _ in range(120):
        p = int(rng.integers(0, 560))
        r = list(genome[p:p + int(rng.integers(0, 40))])
        for i in range(len(r)):
            if rng.random() < 0.03:
                r[i] = "ACGTN"[int(rng.integers(0, 5))]
        reads.append("".join(r))
    # a table of some of the reads' k-mers with random counters
    cand = sorted({brute.encode(brute.canonical(w)) for r in reads for w in brute.windows(r, k)})
    pick = [x for x in cand if rng.random() < 0.6]
    table = {x: tuple(int(v) for v in rng.integers(0, 6, nc)) for x in pick}
    keys = np.array(sorted(table), np.uint64)
    counts = np.array([table[int(x)] for x in keys], np.uint32).reshape(-1, nc)
    b, o = _pack(reads)
    got = oracle.filter_reads(k, nc, keys, counts, b, o, tmin, nmax)
    assert got.tolist() == brute.filter_reads(table, reads, k, tmin, nmax, n_counters=nc)


def test_filter_without_threshold_selects_table_windows():
    rng = np.random.default_rng(5)
    genome = "".join(rng.choice(list("ACGT"), 2000))
    reads = [genome[p:p + 80] for p in rng.integers(0, 1900, 300)]
    b, o = _pack(reads)
    tags = np.array([i % 2 for i in range(len(reads))], np.uint8)
    p = oracle.Params(k=15, n_counters=2, m_log2=18, h=3, block_log2=12, seed=5)
    res = oracle.count(p, b, o, tags=tags, want_bloom=False)
    present = set(int(x) for x in res.keys)
    want = [sum(brute.encode(brute.canonical(w)) in present for w in brute.windows(r, 15))
            for r in reads]
    # tumour >= 0 and normal <= max: every window is selected
    assert oracle.filter_reads(15, 2, res.keys, res.counts, b, o, 0, 2**32 - 1).tolist() == \
        [len(r) - 14 for r in reads]
    # tumour >= 1 with no normal cap, on a table whose tumour counter is the
    # total: exactly the windows whose k-mer is in the table
    tot = res.counts.sum(axis=1, dtype=np.uint32)
    both = np.stack([np.zeros_like(tot), tot], axis=1)
    assert oracle.filter_reads(15, 2, res.keys, both, b, o, 1, 2**32 - 1).tolist() == want
