"""Pins of the CPU oracle against what the paper and the mathematics fix.

These run without a GPU.  Each test targets a plausible mistake in the oracle:
bit order or missing complement (worked example), windows spanning reads or an
off-by-one in the window count (closed forms), wrong Bloom saturation or
missing de-duplication of bit positions (brute force with tiny blocks), order
dependence (shuffles), reverse-complement handling (strand flips).
"""
import random

import numpy as np
import pytest

import oracle
from oracle import brute

M64 = (1 << 64) - 1


def pack_reads(reads):
    offs = np.zeros(len(reads) + 1, dtype=np.uint64)
    for i, r in enumerate(reads):
        offs[i + 1] = offs[i] + len(r)
    data = "".join(reads).encode()
    return np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(0, np.uint8), offs


def rand_reads(rng, n, lmin, lmax, nfrac=0.0, alphabet="ACGT"):
    out = []
    for _ in range(n):
        L = rng.randint(lmin, lmax)
        s = []
        for _ in range(L):
            if nfrac and rng.random() < nfrac:
                s.append(rng.choice("NnRX"))
            else:
                s.append(rng.choice(alphabet))
        out.append("".join(s))
    return out


def table_of(res):
    return {int(k): tuple(int(c) for c in cs) for k, cs in zip(res.keys, res.counts)}


def bits_of(words):
    out = set()
    for w, v in enumerate(words):
        v = int(v)
        while v:
            b = v & -v
            out.add(w * 64 + b.bit_length() - 1)
            v ^= b
    return out


# ---------------------------------------------------------------- the hash

def test_mix64_published_vectors(golden):
    rows = golden("splitmix64_seed0.txt")
    for i, (hexv,) in enumerate(rows):
        want = int(hexv, 16)
        z = ((i + 1) * brute.GAMMA) & M64
        assert brute.mix64(z) == want
        assert oracle.mix64(z) == want


def test_mix64_c_matches_python():
    rng = random.Random(5)
    for _ in range(20000):
        z = rng.getrandbits(64)
        assert oracle.mix64(z) == brute.mix64(z)


def test_mix64_no_collisions_small_range():
    vals = {brute.mix64(i) for i in range(200000)}
    assert len(vals) == 200000


# -------------------------------------------------------- worked examples

def test_worked_example(golden):
    rows = golden("worked_example.txt")
    read = rows[0][1]
    k = int(rows[1][1])
    want = [(r[1], r[3], int(r[5], 16)) for r in rows[2:]]
    assert len(want) == len(read) - k + 1
    p = oracle.Params(k=k, m_log2=10, h=2, block_log2=4, seed=1)
    b, o = pack_reads([read])
    keys = oracle.enumerate_keys(p, b, o)
    assert [int(v) >> 1 for v in keys] == [c for _, _, c in want]
    for i, (win, canon, code) in enumerate(want):
        assert read[i:i + k] == win
        assert brute.canonical(win) == canon
        assert brute.encode(canon) == code


def test_amplification(golden):
    rows = dict((r[0], int(r[1])) for r in golden("amplification.txt"))
    rng = random.Random(3)
    read = "".join(rng.choice("ACGT") for _ in range(rows["read_len"]))
    p = oracle.Params(k=rows["k"], m_log2=12, h=2, block_log2=6)
    b, o = pack_reads([read])
    res = oracle.count(p, b, o)
    assert res.stats["n_valid"] == rows["kmers"]
    assert res.stats["n_valid"] * 8 == rows["bytes"]


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", [1, 2, 7, 13, 31])
def test_window_count_closed_form(k):
    rng = random.Random(k)
    reads = rand_reads(rng, 300, 0, 60)
    p = oracle.Params(k=k, m_log2=14, h=3, block_log2=8, seed=9)
    b, o = pack_reads(reads)
    res = oracle.count(p, b, o)
    assert res.stats["n_valid"] == sum(max(0, len(r) - k + 1) for r in reads)


def test_windows_never_span_reads():
    # Each read alone has no valid window; concatenated they would.
    reads = ["ACGT", "ACGT", "ACG"]
    p = oracle.Params(k=5, m_log2=10, h=2, block_log2=5)
    b, o = pack_reads(reads)
    assert oracle.count(p, b, o).stats["n_valid"] == 0


@pytest.mark.parametrize("base,code", [("A", 0), ("T", 0), ("C", None), ("G", None)])
def test_homopolymer(base, code):
    k, L = 21, 80
    p = oracle.Params(k=k, m_log2=12, h=3, block_log2=6)
    b, o = pack_reads([base * L])
    res = oracle.count(p, b, o)
    # A..A and T..T are each other's reverse complement -> key 0.
    # C..C (code sum 4^j) is smaller than its reverse complement G..G.
    want = code if code is not None else sum(4 ** j for j in range(k))
    assert table_of(res) == {want: (L - k + 1,)}
    assert res.stats["sum_counts"] == L - k + 1


def test_invalid_bytes_break_windows():
    # lowercase, N and IUPAC codes all invalidate the windows covering them
    reads = ["ACGTAcGTACGT", "ACGTANGTACGT", "ACGTARGTACGT"]
    p = oracle.Params(k=4, m_log2=10, h=2, block_log2=5)
    b, o = pack_reads(reads)
    res = oracle.count(p, b, o)
    # each read has 9 windows, 4 of which cover position 5
    assert res.stats["n_valid"] == 3 * (9 - 4)


# ------------------------------------------------------------ brute force

PARAM_SETS = [
    # k, m_log2, h, block_log2, seed, min_count, n_counters
    (5, 10, 3, 4, 11, 2, 1),
    (7, 12, 4, 12, 12, 2, 1),
    (9, 9, 2, 1, 13, 2, 1),      # 2-bit blocks: duplicated positions in S(x)
    (3, 8, 8, 2, 14, 2, 1),      # h > block size: heavy duplication
    (11, 16, 3, 6, 15, 3, 1),
    (8, 11, 4, 5, 16, 2, 2),     # joint normal/tumour counters
    (31, 20, 4, 19, 17, 2, 1),
    (1, 6, 2, 3, 18, 2, 1),
    (2, 6, 3, 6, 19, 2, 2),
]


@pytest.mark.parametrize("k,m_log2,h,bl,seed,minc,nc", PARAM_SETS)
def test_oracle_matches_brute_force(k, m_log2, h, bl, seed, minc, nc):
    rng = random.Random(seed * 1000 + k)
    # a small alphabet of reads sampled from a short genome gives repeats
    genome = "".join(rng.choice("ACGT") for _ in range(400))
    reads = []
    for _ in range(120):
        L = rng.randint(0, 40)
        st = rng.randint(0, len(genome) - L)
        s = list(genome[st:st + L])
        for j in range(L):
            if rng.random() < 0.02:
                s[j] = rng.choice("ACGTN")
        r = "".join(s)
        if rng.random() < 0.5:
            r = brute.revcomp(r.replace("N", "A")) if "N" not in r else r[::-1]
        reads.append(r)
    tags = [rng.randint(0, nc - 1) for _ in reads]
    p = oracle.Params(k=k, m_log2=m_log2, h=h, block_log2=bl, seed=seed, min_count=minc,
                      n_counters=nc)
    b, o = pack_reads(reads)
    res = oracle.count(p, b, o, tags=np.array(tags, np.uint8) if nc > 1 else None)
    t, b1, b2, st = brute.count(reads, k, m_log2, h, bl, seed, minc,
                                tags=tags if nc > 1 else None, n_counters=nc)
    assert table_of(res) == t
    assert bits_of(res.b1) == b1
    assert bits_of(res.b2) == b2
    assert res.stats == st


def test_bloom_bits_match_brute():
    rng = random.Random(21)
    for (k, m_log2, h, bl, seed, _, _) in PARAM_SETS:
        p = oracle.Params(k=k, m_log2=m_log2, h=h, block_log2=bl, seed=seed)
        for _ in range(200):
            x = rng.getrandbits(2 * k)
            assert set(oracle.bloom_bits(p, x)) == brute.bloom_set(x, m_log2, h, bl, seed)


def test_bloom_positions_hand_worked(golden):
    """S(x) against positions worked by hand from the published SplitMix64
    outputs (tests/golden/bloom_positions.txt): a wrong field of the hash (a
    or b), a wrong step, a missed reduction modulo the block or a wrong block
    prefix changes one of them."""
    rows = golden("bloom_positions.txt")
    assert len(rows) == 7
    for kind, seed, key, m, bl, h, want in rows:
        p = oracle.Params(k=31, m_log2=int(m), h=int(h), block_log2=int(bl), seed=int(seed, 16))
        x = int(key, 16)
        got = oracle.bloom_bits(p, x)
        ref = brute.bloom_set(x, int(m), int(h), int(bl), int(seed, 16))
        assert set(got) == ref
        if kind == "positions":
            vals = [int(v) for v in want.split(",")]
            # distinct positions in hash order (S(x) is a set)
            assert got == list(dict.fromkeys(vals))
        else:
            assert {q >> int(bl) for q in got} == {int(want)}


def test_oracle_rejects_blocks_wider_than_half_a_hash():
    """a and b are two block-sized fields of one 64-bit hash, so a Bloom block
    of more than 2^32 bits has no defined positions: the oracle refuses it."""
    import numpy as np
    p = oracle.Params(k=5, m_log2=36, h=4, block_log2=33, seed=1)
    with pytest.raises(ValueError):
        oracle.bloom_bits(p, 12345)
    with pytest.raises(ValueError):
        oracle.count(p, np.frombuffer(b"ACGTACGTAC", np.uint8), np.array([0, 10], np.uint64))
    ok = oracle.Params(k=5, m_log2=36, h=4, block_log2=32, seed=1)
    assert set(oracle.bloom_bits(ok, 12345)) == brute.bloom_set(12345, 36, 4, 32, 1)


# ---------------------------------------------------------------- invariants

def _sim_reads(seed, n, L, err=0.01):
    rng = random.Random(seed)
    genome = "".join(rng.choice("ACGT") for _ in range(3000))
    out = []
    for _ in range(n):
        st = rng.randint(0, len(genome) - L)
        s = list(genome[st:st + L])
        for j in range(L):
            if rng.random() < err:
                s[j] = rng.choice("ACGT")
        r = "".join(s)
        out.append(brute.revcomp(r) if rng.random() < 0.5 else r)
    return out


def test_reverse_complement_invariance():
    reads = _sim_reads(2, 400, 60)
    p = oracle.Params(k=15, m_log2=14, h=3, block_log2=7, seed=3)
    r1 = oracle.count(p, *pack_reads(reads))
    r2 = oracle.count(p, *pack_reads([brute.revcomp(r) for r in reads]))
    assert table_of(r1) == table_of(r2)
    assert np.array_equal(r1.b1, r2.b1) and np.array_equal(r1.b2, r2.b2)
    assert r1.stats == r2.stats


def test_order_invariance():
    reads = _sim_reads(4, 400, 60)
    p = oracle.Params(k=13, m_log2=13, h=4, block_log2=6, seed=5)
    r1 = oracle.count(p, *pack_reads(reads))
    rng = random.Random(8)
    sh = reads[:]
    rng.shuffle(sh)
    r2 = oracle.count(p, *pack_reads(sh))
    assert table_of(r1) == table_of(r2)
    assert np.array_equal(r1.b1, r2.b1) and np.array_equal(r1.b2, r2.b2)
    assert r1.stats == r2.stats


def test_sum_invariant_and_no_false_negatives():
    reads = _sim_reads(6, 500, 80)
    p = oracle.Params(k=21, m_log2=12, h=3, block_log2=5, seed=7)
    b, o = pack_reads(reads)
    res = oracle.count(p, b, o)
    keys = oracle.enumerate_keys(p, b, o) >> np.uint64(1)
    uniq, cnt = np.unique(keys, return_counts=True)
    assert int(cnt.sum()) == res.stats["n_valid"]
    assert res.stats["n_distinct"] == uniq.size
    b2 = bits_of(res.b2)
    for x in res.keys[:500]:
        assert set(oracle.bloom_bits(p, int(x))) <= b2
    # every key of the table passes, so N_pass = sum over table + F
    assert res.stats["n_pass"] == res.stats["sum_counts"] + res.stats["fp_singletons"]
    assert bits_of(res.b2) <= bits_of(res.b1)


def test_saturated_bloom_passes_every_singleton():
    reads = _sim_reads(7, 200, 50, err=0.05)
    p = oracle.Params(k=17, m_log2=2, h=3, block_log2=2, seed=1)
    res = oracle.count(p, *pack_reads(reads))
    assert res.stats["b2_pop"] == 4
    singletons = res.stats["n_distinct"] - res.stats["entries"]
    assert res.stats["fp_singletons"] == singletons
    assert res.stats["n_pass"] == res.stats["n_valid"]


def test_sparse_bloom_has_no_false_positives():
    reads = _sim_reads(9, 100, 50, err=0.05)
    p = oracle.Params(k=17, m_log2=36, h=4, block_log2=19, seed=2)
    res = oracle.count(p, *pack_reads(reads), want_bloom=False)
    assert res.stats["fp_singletons"] == 0
    assert res.stats["n_pass"] == res.stats["sum_counts"]


def test_min_count_threshold():
    reads = _sim_reads(10, 300, 40)
    p2 = oracle.Params(k=11, m_log2=12, h=3, block_log2=6, seed=4, min_count=2)
    p4 = oracle.Params(k=11, m_log2=12, h=3, block_log2=6, seed=4, min_count=4)
    r2 = oracle.count(p2, *pack_reads(reads))
    r4 = oracle.count(p4, *pack_reads(reads))
    t2 = table_of(r2)
    assert table_of(r4) == {x: c for x, c in t2.items() if c[0] >= 4}
    assert r2.stats["fp_singletons"] == r4.stats["fp_singletons"]


def test_joint_counts_sum_to_single():
    reads = _sim_reads(11, 300, 50)
    rng = random.Random(1)
    tags = np.array([rng.randint(0, 1) for _ in reads], np.uint8)
    p1 = oracle.Params(k=15, m_log2=13, h=3, block_log2=7, seed=6)
    p2 = oracle.Params(k=15, m_log2=13, h=3, block_log2=7, seed=6, n_counters=2)
    b, o = pack_reads(reads)
    r1 = oracle.count(p1, b, o)
    r2 = oracle.count(p2, b, o, tags=tags)
    assert {x: (sum(c),) for x, c in table_of(r2).items()} == table_of(r1)
    assert np.array_equal(r1.b1, r2.b1) and np.array_equal(r1.b2, r2.b2)
    # counter split equals counting each sample alone
    for t in (0, 1):
        sub = [r for r, g in zip(reads, tags) if g == t]
        alone = oracle.count(oracle.Params(k=15, m_log2=13, h=3, block_log2=7, seed=6,
                                           min_count=2), *pack_reads(sub))
        for x, c in table_of(r2).items():
            if c[t] >= 2:
                assert table_of(alone)[x] == (c[t],)


def test_sampled_counts_and_hits_match_full():
    reads = _sim_reads(12, 500, 70)
    p = oracle.Params(k=19, m_log2=12, h=3, block_log2=6, seed=8)
    b, o = pack_reads(reads)
    res = oracle.count(p, b, o)
    full = dict(zip(oracle.enumerate_keys(p, b, o) >> np.uint64(1), [None] * 1))
    keys = np.concatenate([res.keys[::7], np.array([0, 12345], np.uint64)])
    ks, cs, nv = oracle.sample_counts(p, b, o, keys, threads=3)
    assert nv == res.stats["n_valid"]
    t = table_of(res)
    enum = oracle.enumerate_keys(p, b, o) >> np.uint64(1)
    for x, c in zip(ks, cs):
        assert int(c[0]) == int(np.count_nonzero(enum == x))
        if int(x) in t:
            assert t[int(x)] == (int(c[0]),)
    b1, b2 = bits_of(res.b1), bits_of(res.b2)
    # every block sampled, then bits of two blocks only (keys of the other
    # blocks are skipped by the scan and must not change the result)
    for bits in (np.arange(0, 1 << 12, 5, dtype=np.uint64),
                 np.concatenate([np.arange(3 * 64, 4 * 64, dtype=np.uint64),
                                 np.arange(40 * 64 + 1, 41 * 64, 3, dtype=np.uint64)])):
        bs, hs = oracle.sample_hits(p, b, o, bits, threads=2)
        assert np.array_equal(bs, np.unique(bits))
        for bit, hcount in zip(bs, hs):
            assert (int(hcount) >= 1) == (int(bit) in b1)
            assert (int(hcount) >= 2) == (int(bit) in b2)
    del full


# ------------------------------------------------------ value-range passes

RANGE_CASES = [  # (k, m_log2, h, bl, nc, qbits, threads, keep_singles)
    (31, 20, 4, 12, 1, 0, 1, True),
    (31, 20, 4, 12, 1, 3, 4, True),
    (21, 18, 3, 18, 2, 4, 3, False),
    (13, 16, 2, 5, 1, 6, 8, True),
    (5, 12, 4, 2, 2, 10, 8, False),   # qbits = 2k: one key per range
    (3, 10, 3, 3, 1, 2, 8, True),     # more threads than ranges
    (31, 24, 4, 16, 2, 5, 7, True),
]


@pytest.mark.parametrize("k,m_log2,h,bl,nc,qbits,threads,keep", RANGE_CASES)
def test_value_range_passes_equal_the_full_count(k, m_log2, h, bl, nc, qbits, threads, keep):
    """or_count_ranges (value-range passes, threads, atomic Bloom updates,
    the screen after the last pass) gives the table, both levels and every
    statistic of the single sort, also with fewer threads than ranges (several
    passes) and with a second round of passes for the screen."""
    import numpy as np
    from kc_cases import pack_reads, random_reads
    reads = random_reads(100 + k, 1500, 5, 160, genome_len=3000)
    b, o = pack_reads(reads)
    tags = np.array([i % 2 for i in range(len(reads))], np.uint8) if nc == 2 else None
    p = oracle.Params(k=k, n_counters=nc, m_log2=m_log2, h=h, block_log2=bl, seed=k * 7 + 1)
    ref = oracle.count(p, b, o, tags=tags)
    got = oracle.count_ranges(p, b, o, tags=tags, qbits=qbits, threads=threads, keep_singles=keep)
    assert np.array_equal(got.keys, ref.keys)
    assert np.array_equal(got.counts, ref.counts)
    assert np.array_equal(got.b1, ref.b1) and np.array_equal(got.b2, ref.b2)
    assert got.stats == ref.stats


def test_value_range_passes_match_brute_force():
    """The range passes against the string-level brute force directly."""
    import numpy as np
    from kc_cases import pack_reads, random_reads
    reads = random_reads(7, 300, 8, 60, genome_len=400)
    b, o = pack_reads(reads)
    p = oracle.Params(k=9, m_log2=10, h=3, block_log2=4, seed=5)
    got = oracle.count_ranges(p, b, o, qbits=5, threads=4)
    t, b1, b2, st = brute.count(reads, 9, 10, 3, 4, 5)
    assert {int(x): (int(c),) for x, c in zip(got.keys, got.counts[:, 0])} == t
    bits = lambda v: {w * 64 + j for w in range(v.size) for j in range(64) if (int(v[w]) >> j) & 1}
    assert bits(got.b1) == b1 and bits(got.b2) == b2
    assert got.stats == st


def test_streamed_table_digest_equals_the_whole_table_digest():
    """Value-range passes handing each range's table to a callback (and
    screening in a second sweep) give the digest and statistics of the
    gathered table."""
    import numpy as np
    import synth
    from digest import TableDigest, table_digests
    w = synth.WORKLOADS["plain_1mbp"]
    g = w.make_genome()
    b, o = w.make_reads(g, n=6000)
    p = oracle.Params(k=w.k, m_log2=w.bloom_bits_log2, h=w.bloom_hashes,
                      block_log2=w.bloom_block_log2, seed=w.seed)
    full = oracle.count(p, b, o, want_bloom=True)
    td = TableDigest(w.k)
    seen = []
    part = oracle.count_ranges(p, b, o, qbits=6, threads=3, keep_singles=False,
                               on_range=lambda q, k, c: (seen.append(q), td.update(k, c)))
    assert seen == sorted(seen) and len(seen) == 64
    assert part.keys.size == 0
    assert td.result() == table_digests(full.keys, full.counts, w.k)
    assert part.stats == full.stats
    assert np.array_equal(part.b1, full.b1) and np.array_equal(part.b2, full.b2)


def test_digest_file_reproduces_from_the_oracle():
    """The committed whole-output digest of the 1 Mbp workload is what the
    oracle gives now (the GPU tests compare against these files)."""
    import os
    import numpy as np
    import synth
    from digest import read_digest_file, table_digests, words_digest
    from conftest import GOLDEN
    w = synth.WORKLOADS["plain_1mbp"]
    g = w.make_genome()
    b, o = w.make_reads(g)
    p = oracle.Params(k=w.k, m_log2=w.bloom_bits_log2, h=w.bloom_hashes,
                      block_log2=w.bloom_block_log2, seed=w.seed)
    res = oracle.count(p, b, o)
    want = read_digest_file(os.path.join(GOLDEN, "digest_plain_1mbp.txt"))
    got = table_digests(res.keys, res.counts, w.k)
    assert got["sha256"] == want["sha256"]
    assert [tuple(r) for r in got["ranges"]] == want["ranges"]
    assert words_digest(res.b1) == want["b1"] and words_digest(res.b2) == want["b2"]
    assert want["stats"]["fp_singletons"] == res.stats["fp_singletons"]
    assert want["stats"]["n_pass"] == res.stats["n_pass"]
    assert int(np.unpackbits(res.b1.view(np.uint8)).sum()) == want["stats"]["b1_popcount"]


def test_sparse_bloom_output_is_the_nonzero_words():
    """want_bloom="sparse" lists exactly the nonzero level-1 words and both
    levels there (the GPU tests of filters of 2^33 bits and more compare
    these words and the popcounts)."""
    import numpy as np
    from kc_cases import pack_reads, random_reads
    reads = random_reads(9, 500, 20, 120, genome_len=1500)
    b, o = pack_reads(reads)
    p = oracle.Params(k=15, m_log2=22, h=4, block_log2=10, seed=4)
    full = oracle.count(p, b, o)
    for fn in (oracle.count, lambda *a, **kw: oracle.count_ranges(*a, threads=3, **kw)):
        sp = fn(p, b, o, want_bloom="sparse")
        nz = np.flatnonzero(full.b1)
        assert np.array_equal(sp.touched, nz)
        assert np.array_equal(sp.t1, full.b1[nz]) and np.array_equal(sp.t2, full.b2[nz])
        assert not full.b2[full.b1 == 0].any()
        assert sp.stats == full.stats
