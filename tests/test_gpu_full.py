"""Full-size parity on the 100 Mbp / 10M-read workload, in the configuration
bench.py times.  The whole table is too large to sort on the host, so the
oracle computes sampled outputs exactly (threaded scans over every window):
counts of sampled keys and saturating hits of sampled Bloom bits.  Properties
that hold at any size are checked on the full outputs.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from conftest import GOLDEN
from digest import STAT_KEYS, read_digest_file, table_digests, words_digest
from kc_cases import (gpu_table_sorted, note, oracle_params, to_device, workload_chunks,
                      workload_config)
from oracle import brute

pytestmark = pytest.mark.gpu


def _popcount(words):
    v = words.view(np.uint8)
    return int(np.unpackbits(v).sum())


@pytest.mark.parametrize("name", ["plain_1mbp", "plain_100mbp"])
def test_whole_output_digest(name):
    """The whole output at full size, in the configuration bench.py times:
    every statistic, the sorted table (SHA-256 as a whole and per value range)
    and both Bloom levels (SHA-256 of every word) against the digest that
    tests/golden/make_digests.py wrote from the CPU oracle's value-range
    passes over every window."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: %s full size, whole-output digest" % name)
    want = read_digest_file(os.path.join(GOLDEN, "digest_%s.txt" % name))
    w, _, b, o = workload_chunks(name)
    cfg = workload_config(w)
    db, do = to_device(b, o)
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        st = c.finalize()
        keys, counts = c.export()
        b1, b2 = c.export_bloom()
    for key in STAT_KEYS:
        assert st[key] == want["stats"][key], (key, st[key], want["stats"][key])
    ks, cs = gpu_table_sorted(keys, counts)
    got = table_digests(ks, cs, w.k)
    for q, (g, r) in enumerate(zip(got["ranges"], want["ranges"])):
        assert tuple(g) == tuple(r), ("value range", q, g, r)
    assert got["sha256"] == want["sha256"]
    assert words_digest(b1) == want["b1"]
    assert words_digest(b2) == want["b2"]


def test_plain_100mbp_sampled_parity():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: plain_100mbp full size (1e7 reads x 100 bp), sampled parity")
    w, _, b, o = workload_chunks("plain_100mbp")
    cfg = workload_config(w)
    db, do = to_device(b, o)
    rng = np.random.default_rng(2024)
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        st = c.finalize()
        keys, counts = c.export()
        b1, b2 = c.export_bloom()
        # sampled keys: from the table, from random windows of the reads, random codes
        from_table = keys[rng.integers(0, keys.size, 3000)]
        wins = []
        starts = rng.integers(0, w.n_reads, 4000)
        for r in starts:
            lo = int(o[r])
            j = int(rng.integers(0, 100 - w.k + 1))
            s = bytes(b[lo + j:lo + j + w.k]).decode()
            if all(ch in "ACGT" for ch in s):
                wins.append(brute.encode(brute.canonical(s)))
        rand = rng.integers(0, 1 << (2 * w.k), 1000, dtype=np.uint64)
        sample = np.unique(np.concatenate([from_table, np.array(wins, np.uint64), rand]))
        q = torch.from_numpy(sample.view(np.int64)).cuda()
        got = c.query(q).cpu().numpy().astype(np.uint32)[:, 0]
        # Filter lookup over all windows: with count >= min_count selected, the
        # selected windows are exactly the occurrences of table k-mers
        sel = c.filter_reads(db, do, cfg.min_count, 0).to(torch.int64)
        assert int(sel.sum().item()) == st["sum_counts"]
        # ... and with no threshold every window is selected
        every = c.filter_reads(db, do, 0, 0xFFFFFFFF).to(torch.int64)
        assert int(every.sum().item()) == st["n_valid"]
        # stem items hold every table k-mer once (counts stay below 2^16 here)
        stems, items = c.export_stems()
        it = items.to(torch.int32) & 0xFFFF
        assert int((it > 0).sum().item()) == st["entries"]
        assert int(it.sum().item()) == st["sum_counts"]
        del stems, items, it
    note("sample keys: %d; oracle scan over all windows" % sample.size)
    p = oracle_params(cfg)
    ks, cs, nv = oracle.sample_counts(p, b, o, sample, threads=16)
    assert np.array_equal(ks, sample)
    want = np.where(cs[:, 0] >= cfg.min_count, cs[:, 0], 0)
    assert nv == st["n_valid"]
    assert np.array_equal(got, want)
    # the exported table agrees with the sample
    order = np.argsort(keys)
    sk, sc = keys[order], counts[order, 0]
    at = np.searchsorted(sk, sample)
    present = (at < sk.size) & (sk[np.minimum(at, sk.size - 1)] == sample)
    assert np.array_equal(present, want > 0)
    assert np.array_equal(sc[at[present]], want[present])

    # sampled Bloom bits: random positions plus the positions of sampled keys
    m = 1 << cfg.bloom_bits_log2
    bits = list(rng.integers(0, m, 3000, dtype=np.uint64))
    for x in sample[:300]:
        bits += oracle.bloom_bits(p, int(x))
    bs, hs = oracle.sample_hits(p, b, o, np.array(bits, np.uint64), threads=16)
    g1 = (b1[bs >> np.uint64(6)] >> (bs & np.uint64(63))) & np.uint64(1)
    g2 = (b2[bs >> np.uint64(6)] >> (bs & np.uint64(63))) & np.uint64(1)
    assert np.array_equal(g1.astype(bool), hs >= 1)
    assert np.array_equal(g2.astype(bool), hs >= 2)

    # properties that hold at any size
    assert keys.size == st["entries"] == np.unique(keys).size
    assert int(counts.sum()) == st["sum_counts"]
    assert counts.min() >= cfg.min_count
    assert st["n_pass"] == st["sum_counts"] + st["fp_singletons"]
    assert _popcount(b1) == st["b1_popcount"] and _popcount(b2) == st["b2_popcount"]
    assert st["b2_popcount"] <= st["b1_popcount"]
    assert int(keys.max()) < (1 << (2 * cfg.k))
    note("entries %d, F %d, overflow keys %d" % (st["entries"], st["fp_singletons"],
                                                st["overflow_keys"]))


def test_plain_100mbp_most_keys_in_the_overflow_table():
    """The same workload with 2^17 partition tables of 128 slots (1.7·10^7
    slots in all): about 8·10^7 of the 9.8·10^7 counted keys do not fit and go
    to the overflow table, which finalize grows more than once.  Partitioning
    and table size change no result: statistics, exported table and queries
    equal those of the configuration bench.py times."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: plain_100mbp full size, 2^17 partitions of 128 slots (overflow-heavy) "
         "against 2^16 partitions of 3840")
    w, _, b, o = workload_chunks("plain_100mbp")
    base = workload_config(w)
    heavy = workload_config(w, partitions_log2=17, table_slots=128)
    db, do = to_device(b, o)
    rng = np.random.default_rng(77)
    out = []
    for cfg in (base, heavy):
        with kc.KmerCounter(cfg) as c:
            c.insert_reads(db, do)
            st = c.finalize()
            keys, counts = c.export()
            if not out:
                sample = np.concatenate([keys[rng.integers(0, keys.size, 20000)],
                                         rng.integers(0, 1 << (2 * w.k), 5000, dtype=np.uint64)])
                q = torch.from_numpy(sample.view(np.int64)).cuda()
            got = c.query(q).cpu().numpy()
        note("partitions 2^%d: entries %d, overflow keys %d, retries %d"
             % (st["partitions_log2"], st["entries"], st["overflow_keys"], st["retries"]))
        out.append((st, keys, counts, got))
    (s0, k0, c0, q0), (s1, k1, c1, q1) = out
    assert s1["overflow_keys"] > s1["entries"] // 2
    assert s1["retries"] >= 1
    for key in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons",
                "passed_distinct", "b1_popcount", "b2_popcount"):
        assert s1[key] == s0[key], key
    o0, o1 = np.argsort(k0), np.argsort(k1)
    assert np.array_equal(k0[o0], k1[o1])
    assert np.array_equal(c0[o0], c1[o1])
    assert np.array_equal(q0, q1)


def test_batched_200mbp_whole_output_digest():
    """The batched workload at full size (256 chunks, 7.08·10^7 reads of
    100-250 bp, 1.03·10^10 k-mers, 2^35-bit levels) as one kc_count_batch
    graph launch with the configuration the autotuner picks there (2^18
    partitions, first-level split 9; result-neutral): every statistic, the
    sorted table (whole and per value range) and both levels against the
    digest of the oracle's value-range passes over the same read stream."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: batched_200mbp full size (256 chunks), one graph launch, whole-output digest")
    want = read_digest_file(os.path.join(GOLDEN, "digest_batched_200mbp.txt"))
    import synth
    w = synth.WORKLOADS["batched_200mbp"]
    genome = w.make_genome(threads=16)
    sizes = w.chunk_plan()
    dev = []
    for i in range(sizes.size):
        b, o = w.make_chunk(genome, sizes, i, threads=16)
        dev.append(to_device(b, o))
    del genome
    note("chunks on the device: %d reads, %d bases" % (int(sizes.sum()),
                                                        sum(int(b.numel()) for b, _ in dev)))
    cfg = workload_config(w, partitions_log2=18, scatter_bits=9)
    with kc.KmerCounter(cfg) as c:
        st = c.count_batch(dev)
        torch.cuda.synchronize()
        del dev
        keys, counts = c.export()
        b1, b2 = c.export_bloom()
    for key in STAT_KEYS:
        assert st[key] == want["stats"][key], (key, st[key], want["stats"][key])
    ks, cs = gpu_table_sorted(keys, counts)
    del keys, counts
    got = table_digests(ks, cs, w.k)
    for q, (g, r) in enumerate(zip(got["ranges"], want["ranges"])):
        assert tuple(g) == tuple(r), ("value range", q, g, r)
    assert got["sha256"] == want["sha256"]
    assert words_digest(b1) == want["b1"]
    assert words_digest(b2) == want["b2"]


@pytest.mark.parametrize("budget_gib", [0, 24])
def test_spill_3gbp_whole_output_digest(budget_gib):
    """The 3 Gbp workload at full size (2·10^8 reads of 100 bp, 1.4·10^10
    k-mers, 2^36-bit levels, 2^20 partitions), inserted as 8 consecutive
    slices of the read stream as bench.py does, with its 64 GB table budget
    (every table resident) and with a 24 GiB budget (about half the tables
    counted in waves and spilled to pinned host memory, exported from there):
    every statistic, the sorted table (whole and per value range) and both
    levels against the digest of the oracle's streamed value-range passes.
    The 2.6·10^9-entry table is sorted on the device one value range at a
    time."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth
    from digest import TableDigest
    note("case: spill_3gbp full size (8 inserts of 2.5e7 reads x 100 bp), table budget %s, "
         "whole-output digest" % ("%d GiB" % budget_gib if budget_gib else "of the workload"))
    want = read_digest_file(os.path.join(GOLDEN, "digest_spill_3gbp.txt"))
    w = synth.WORKLOADS["spill_3gbp"]
    genome = w.make_genome(threads=16)
    per = w.n_reads
    while per * w.lmax >= 1 << 32:
        per = (per + 1) // 2
    cfg = workload_config(w, **({"hbm_table_budget_bytes": budget_gib << 30} if budget_gib else {}))
    with kc.KmerCounter(cfg) as c:
        for f in range(0, w.n_reads, per):
            b, o = w.make_reads(genome, first=f, n=min(per, w.n_reads - f), threads=16)
            db, do = to_device(b, o)
            del b, o
            c.insert_reads(db, do)
            torch.cuda.synchronize()
            del db, do
            note("inserted reads %d..%d" % (f, min(f + per, w.n_reads) - 1))
        del genome
        st = c.finalize()
        for key in STAT_KEYS:
            assert st[key] == want["stats"][key], (key, st[key], want["stats"][key])
        if budget_gib:
            assert st["spilled_partitions"] > 0
            note("spilled %d partitions, %.1f GB" % (st["spilled_partitions"],
                                                     st["spilled_bytes"] / 1e9))
        b1, b2 = c.export_bloom()
        assert words_digest(b1) == want["b1"]
        assert words_digest(b2) == want["b2"]
        del b1, b2
        note("statistics and both levels equal; exporting %d entries" % st["entries"])
        keys, counts = c.export()
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    del keys
    cd = torch.from_numpy(np.ascontiguousarray(counts).view(np.int32)).cuda()
    del counts
    td = TableDigest(w.k)
    shift = 2 * w.k - td.rb
    step = 1 << 30  # torch's index selection is kept below 2^31 elements per call
    for q in range(1 << td.rb):
        ks, cs = [], []
        for lo in range(0, kd.numel(), step):
            part = kd[lo:lo + step]
            sel = (part >> shift) == q
            ks.append(part[sel])
            cs.append(cd[lo:lo + step][sel])
        kq, cq = torch.cat(ks), torch.cat(cs)
        order = torch.argsort(kq)  # keys < 2^62: signed order is unsigned order
        td.update(kq[order].cpu().numpy().view(np.uint64),
                  cq[order].cpu().numpy().view(np.uint32))
        del ks, cs, kq, cq, order
    del kd, cd
    got = td.result()
    for q, (g, r) in enumerate(zip(got["ranges"], want["ranges"])):
        assert tuple(g) == tuple(r), ("value range", q, g, r)
    assert got["sha256"] == want["sha256"]
