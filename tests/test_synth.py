"""Seeded input generator: determinism, slicing, shapes and rates (CPU only)."""
import numpy as np

import synth

COMP = bytes.maketrans(b"ACGT", b"TGCA")


def test_genome_deterministic_and_uniform():
    a = synth.genome(7, 200_000)
    b = synth.genome(7, 200_000, threads=3)
    c = synth.genome(8, 200_000)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    vals, cnt = np.unique(a, return_counts=True)
    assert bytes(vals) == b"ACGT"
    assert np.all(np.abs(cnt / a.size - 0.25) < 0.01)


def test_reads_slice_equals_whole():
    g = synth.genome(3, 50_000)
    b, o = synth.reads(3, g, 0, 500, 80, 120, 0.02, 0.01)
    b2, o2 = synth.reads(3, g, 200, 100, 80, 120, 0.02, 0.01, threads=2)
    assert np.array_equal(b2, b[int(o[200]):int(o[300])])
    assert np.array_equal(o2, o[200:301] - o[200])
    lens = np.diff(o)
    assert lens.min() >= 80 and lens.max() <= 120


def test_reads_error_and_n_rates():
    g = synth.genome(5, 100_000)
    n, L = 4000, 100
    b, o = synth.reads(5, g, 0, n, L, L, 0.01, 0.001)
    gs = bytes(g)
    mism = ns = tot = 0
    for i in range(n):
        r = bytes(b[i * L:(i + 1) * L])
        # locate the source: exact 20-base anchor on either strand (spurious hits ~1e-7)
        best = None
        for cand in (r, r.translate(COMP)[::-1]):
            pos = gs.find(cand[:20])
            if pos >= 0 and b"N" not in cand[:20]:
                best = (cand, pos)
                break
        if best is None:
            continue
        cand, pos = best
        src = gs[pos:pos + L]
        if len(src) < L:
            continue
        for x, y in zip(cand, src):
            if x == ord("N"):
                ns += 1
            elif x != y:
                mism += 1
            tot += 1
    assert tot > 200_000
    assert abs(mism / tot - 0.01) < 0.002
    assert abs(ns / tot - 0.001) < 0.0004


def test_tumour_mutations():
    g = synth.genome(9, 100_000)
    t = synth.tumour(9, g, 100, 0, 10, 20)
    assert int(np.count_nonzero(g != t)) == 100
    t2 = synth.tumour(9, g, 0, 1, 1000, 1000)
    d = np.nonzero(g != t2)[0]
    assert d.size > 0 and d.max() - d.min() < 1000
    lo = d.min()
    # an inversion is a reverse complement in place: find its exact extent
    for st in range(max(0, d.max() - 999), lo + 1):
        seg = bytes(g[st:st + 1000]).translate(COMP)[::-1]
        if seg == bytes(t2[st:st + 1000]):
            break
    else:
        raise AssertionError("no reverse-complemented segment found")


def test_chunk_sizes_log_uniform():
    c = synth.chunk_sizes(3, 4000, 1e3, 2e6)
    assert c.min() >= 1000 and c.max() <= 2_000_000
    med = np.median(np.log(c.astype(np.float64)))
    assert abs(med - 0.5 * (np.log(1e3) + np.log(2e6))) < 0.3
