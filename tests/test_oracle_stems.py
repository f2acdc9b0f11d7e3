"""Pins of the oracle's stem items (paper Sec. II-A stems, Sec. III-D items
of 16 normal and 16 tumour counts per stem) against the paper's example, a
string-level brute force and invariants of a real count."""
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stem_example.txt")


def test_paper_stem_example():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for r in rows:
        f = dict(zip(r[0::2], r[1::2]))
        kmer = f["kmer"]
        assert kmer[1:-1] == f["stem"]
        stems, items = oracle.stem_items(len(kmer), 1, [brute.encode(kmer)], [7])
        assert stems.tolist() == [brute.encode(f["canonical"])]
        assert items.shape == (1, 2, 16)
        want = np.zeros((2, 16), np.uint16)
        want[0, int(f["slot"])] = 7
        assert np.array_equal(items[0], want)


def _random_table(rng, k, n, n_counters):
    seen = {}
    while len(seen) < n:
        s = "".join(rng.choice(list("ACGT"), k))
        c = brute.canonical(s)
        cs = tuple(int(v) for v in rng.choice([0, 1, 2, 5, 300, 65535, 65536, 1 << 20], n_counters))
        if sum(cs) == 0:
            cs = (2,) + cs[1:]
        seen[c] = cs
    return seen


@pytest.mark.parametrize("k,n_counters", [(3, 1), (4, 2), (5, 1), (8, 2), (12, 2), (21, 1), (31, 2)])
def test_stem_items_match_brute_force(k, n_counters):
    rng = np.random.default_rng(100 + k)
    table = _random_table(rng, k, min(400, 4 ** k // 3), n_counters)
    keys = np.array([brute.encode(s) for s in table], np.uint64)
    counts = np.array([table[s] for s in table], np.uint32).reshape(-1)
    stems, items = oracle.stem_items(k, n_counters, keys, counts)
    want = brute.stem_items(table, k, n_counters)
    assert stems.tolist() == sorted(brute.encode(s) for s in want)
    for i, st in enumerate(stems):
        w = want[brute.decode(int(st), k - 2)]
        for t in range(2):
            row = w[t] if t < n_counters else [0] * 16
            assert items[i, t].tolist() == row, (k, brute.decode(int(st), k - 2), t)


def test_even_k_palindromic_stems_keep_the_kmer_orientation():
    # k = 4: the stem AT is its own reverse complement, so each k-mer keeps
    # its own flanks: AATC (canonical, rc GATT) at slot 4*A + C = 1, the
    # palindrome CATG at slot 4*C + G = 6
    table = {"AATC": (3,), "CATG": (4,)}
    keys = [brute.encode(s) for s in table]
    stems, items = oracle.stem_items(4, 1, keys, [3, 4])
    assert stems.tolist() == [brute.encode("AT")]
    want = np.zeros(16, np.uint16)
    want[1], want[6] = 3, 4
    assert np.array_equal(items[0, 0], want)
    assert brute.stem_items(table, 4) == {"AT": [want.tolist()]}


def test_stem_items_round_trip_a_real_count():
    rng = np.random.default_rng(7)
    genome = "".join(rng.choice(list("ACGT"), 3000))
    reads = []
    for i in range(400):
        p = int(rng.integers(0, 3000 - 90))
        r = genome[p:p + 90]
        reads.append(r if i % 2 else brute.revcomp(r))
    bases = np.frombuffer("".join(reads).encode(), np.uint8)
    offs = np.concatenate([[0], np.cumsum([len(r) for r in reads])]).astype(np.uint64)
    p = oracle.Params(k=21, m_log2=20, h=3, block_log2=14, seed=3)
    res = oracle.count(p, bases, offs)
    stems, items = oracle.stem_items(21, 1, res.keys, res.counts)
    assert int(items.sum()) == int(res.counts.sum())          # no count reaches 2^16
    assert int((items > 0).sum()) == res.keys.size            # one slot per table k-mer
    back = {}
    for st, it in zip(stems, items):
        s = brute.decode(int(st), 19)
        for slot in np.nonzero(it[0])[0]:
            kmer = "ACGT"[slot // 4] + s + "ACGT"[slot % 4]
            back[brute.encode(brute.canonical(kmer))] = int(it[0, slot])
    assert back == {int(x): int(c) for x, c in zip(res.keys, res.counts[:, 0])}
