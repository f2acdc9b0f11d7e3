"""Full-size runs of the 3 Gbp workload (2·10^8 reads × 100 bp, 1.4·10^10
k-mers, 2^36-bit Bloom levels, 2^20 partitions), inserted in eight calls,
once with its 64 GB table budget and once with a 24 GB budget that forces
the spill of partition tables to pinned host memory; and of the batched
workload (256 chunks counted by one graph launch).

Opt-in (set KC_SCALE=1): it needs about 220 GB of HBM, 70 GB of host memory
and ten minutes, most of it the oracle's scan over every window.  The oracle
cannot sort 1.4·10^10 keys on the host, so it computes sampled outputs
exactly: counts of sampled keys and saturating hits of sampled Bloom bits,
each by a scan over all windows of all reads.
"""
import os
import time

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
import synth
from kc_cases import note, oracle_params, to_device, workload_config
from oracle import brute

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not os.environ.get("KC_SCALE"),
                                 reason="full-size runs; set KC_SCALE=1")]

CHUNKS = 8
GB = 1 << 30


def _bits_at(words, bits):
    return ((words[bits >> np.uint64(6)] >> (bits & np.uint64(63))) & np.uint64(1)).astype(bool)


def test_spill_3gbp_sampled_parity():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = synth.WORKLOADS["spill_3gbp"]
    per = w.n_reads // CHUNKS
    t0 = time.time()
    genome = w.make_genome(threads=16)
    chunks = []
    for i in range(CHUNKS):
        chunks.append(w.make_reads(genome, first=i * per, n=per, threads=16))
        note("generated chunk %d/%d (%.0f s)" % (i + 1, CHUNKS, time.time() - t0))
    del genome
    rng = np.random.default_rng(5)
    # sampled keys: windows of random reads of every chunk, plus random codes
    wins = []
    for b, o in chunks:
        for r in rng.integers(0, per, 500):
            j = int(rng.integers(0, w.lmax - w.k + 1))
            s = bytes(b[int(o[r]) + j:int(o[r]) + j + w.k]).decode()
            wins.append(brute.encode(brute.canonical(s)))
    rand = rng.integers(0, 1 << (2 * w.k), 2000, dtype=np.uint64)
    sample = np.unique(np.concatenate([np.array(wins, np.uint64), rand]))

    runs = {}
    for budget in (w.table_budget, 24 * GB):
        cfg = workload_config(w, hbm_table_budget_bytes=budget)
        note("case: spill_3gbp, table budget %d GiB, %d inserts" % (budget // GB, CHUNKS))
        with kc.KmerCounter(cfg) as c:
            torch.cuda.synchronize()
            t1 = time.time()
            for b, o in chunks:
                db, do = to_device(b, o)
                c.insert_reads(db, do)
                del db, do
            st = c.finalize()
            torch.cuda.synchronize()
            wall = time.time() - t1
            q = torch.from_numpy(sample.view(np.int64)).cuda()
            got = c.query(q).cpu().numpy().astype(np.uint32)[:, 0]
            b1 = b2 = None
            if not runs:
                b1, b2 = c.export_bloom()
        note("budget %d GiB: %.2f s wall incl. H2D; stats %s; kernel ms %s" % (
            budget // GB, wall,
            {k: st[k] for k in ("n_valid", "entries", "fp_singletons", "spilled_partitions",
                                "spilled_bytes", "overflow_keys", "table_slots",
                                "partitions_log2")},
            {k: round(v, 1) for k, v in st["kernel_ms"].items() if v}))
        runs[budget] = (st, got, b1, b2)
        torch.cuda.empty_cache()

    st64, got64, b1, b2 = runs[w.table_budget]
    st24, got24, _, _ = runs[24 * GB]
    assert st64["spilled_partitions"] == 0
    per_table = st24["table_slots"] * 12
    kept = (24 * GB) // per_table
    assert st24["spilled_partitions"] == (1 << st24["partitions_log2"]) - kept
    for k in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount",
              "b2_popcount"):
        assert st24[k] == st64[k], k
    assert np.array_equal(got24, got64)
    assert st64["n_valid"] == w.n_reads * (w.lmax - w.k + 1)  # no N bases: closed form

    # sampled Bloom bits: random bits of 48 random blocks plus the bits of 200 sampled keys
    p = oracle_params(workload_config(w))
    blocks = rng.integers(0, 1 << (w.bloom_bits_log2 - w.bloom_block_log2), 48)
    bits = [np.uint64(blk) * np.uint64(1 << w.bloom_block_log2) +
            rng.integers(0, 1 << w.bloom_block_log2, 60, dtype=np.uint64) for blk in blocks]
    bits = list(np.concatenate(bits))
    for x in sample[:200]:
        bits += oracle.bloom_bits(p, int(x))
    bits = np.unique(np.array(bits, np.uint64))

    cnt = np.zeros(sample.size, np.uint64)
    hits = np.zeros(bits.size, np.uint64)
    nv = 0
    for i, (b, o) in enumerate(chunks):
        ks, cs, n = oracle.sample_counts(p, b, o, sample, threads=16)
        assert np.array_equal(ks, sample)
        cnt += cs[:, 0]
        nv += n
        bs, hs = oracle.sample_hits(p, b, o, bits, threads=16)
        hits += hs
        note("oracle scan chunk %d/%d (%.0f s)" % (i + 1, CHUNKS, time.time() - t0))
    want = np.where(cnt >= w.min_count, cnt, 0).astype(np.uint32)
    assert nv == st64["n_valid"]
    assert np.array_equal(got64, want)
    assert np.array_equal(_bits_at(b1, bits), hits >= 1)
    assert np.array_equal(_bits_at(b2, bits), hits >= 2)
    assert st64["n_pass"] == st64["sum_counts"] + st64["fp_singletons"]
    note("sampled parity: %d keys (%d present), %d Bloom bits" % (
        sample.size, int((want > 0).sum()), bits.size))


def test_batched_200mbp_sampled_parity():
    """The batched workload at full size (256 chunks, 7.1·10^7 reads of
    100-250 bp, 1.03·10^10 k-mers, 2^35-bit Bloom levels) in one
    kc_count_batch graph launch, replayed once; sampled exact parity."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = synth.WORKLOADS["batched_200mbp"]
    t0 = time.time()
    genome = w.make_genome(threads=16)
    sizes = w.chunk_plan()
    chunks = [w.make_chunk(genome, sizes, i, threads=16) for i in range(sizes.size)]
    del genome
    note("generated %d chunks, %d reads (%.0f s)" % (len(chunks), int(sizes.sum()), time.time() - t0))
    rng = np.random.default_rng(3)
    wins = []
    for i in rng.integers(0, len(chunks), 40):
        b, o = chunks[i]
        for r in rng.integers(0, o.size - 1, 100):
            lo, hi = int(o[r]), int(o[r + 1])
            j = int(rng.integers(0, hi - lo - w.k + 1))
            wins.append(brute.encode(brute.canonical(bytes(b[lo + j:lo + j + w.k]).decode())))
    rand = rng.integers(0, 1 << (2 * w.k), 2000, dtype=np.uint64)
    sample = np.unique(np.concatenate([np.array(wins, np.uint64), rand]))
    cfg = workload_config(w)
    dev = [to_device(b, o) for b, o in chunks]
    note("case: batched_200mbp, %d chunks in one graph launch, p=%d" % (len(dev), cfg.partitions_log2))
    with kc.KmerCounter(cfg) as c:
        st = c.count_batch(dev)
        c.reset()
        st2 = c.count_batch(dev)  # replay of the captured graph
        note("stats %s; graph ms %.1f / %.1f" % (
            {k: st2[k] for k in ("n_valid", "entries", "fp_singletons", "overflow_keys",
                                 "n_segments")},
            st["kernel_ms"]["graph"], st2["kernel_ms"]["graph"]))
        for k in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount",
                  "b2_popcount"):
            assert st[k] == st2[k], k
        q = torch.from_numpy(sample.view(np.int64)).cuda()
        got = c.query(q).cpu().numpy().astype(np.uint32)[:, 0]
        b1, b2 = c.export_bloom()
    del dev
    p = oracle_params(cfg)
    blocks = rng.integers(0, 1 << (w.bloom_bits_log2 - w.bloom_block_log2), 48)
    bits = [np.uint64(blk) * np.uint64(1 << w.bloom_block_log2) +
            rng.integers(0, 1 << w.bloom_block_log2, 60, dtype=np.uint64) for blk in blocks]
    bits = list(np.concatenate(bits))
    for x in sample[:200]:
        bits += oracle.bloom_bits(p, int(x))
    bits = np.unique(np.array(bits, np.uint64))
    cnt = np.zeros(sample.size, np.uint64)
    hits = np.zeros(bits.size, np.uint64)
    nv = 0
    # the oracle scans every chunk; 32 chunks at a time share one call
    for g0 in range(0, len(chunks), 32):
        part = chunks[g0:g0 + 32]
        b = np.concatenate([x[0] for x in part])
        offs = [np.zeros(1, np.uint64)]
        base = 0
        for bb, oo in part:
            offs.append(oo[1:] + np.uint64(base))
            base += int(oo[-1])
        o = np.concatenate(offs)
        ks, cs, n = oracle.sample_counts(p, b, o, sample, threads=16)
        cnt += cs[:, 0]
        nv += n
        bs, hs = oracle.sample_hits(p, b, o, bits, threads=16)
        hits += hs
        note("oracle scan chunks %d-%d (%.0f s)" % (g0, g0 + len(part) - 1, time.time() - t0))
    want = np.where(cnt >= w.min_count, cnt, 0).astype(np.uint32)
    assert nv == st["n_valid"]
    assert np.array_equal(got, want)
    assert np.array_equal(_bits_at(b1, bits), hits >= 1)
    assert np.array_equal(_bits_at(b2, bits), hits >= 2)
    assert st["n_pass"] == st["sum_counts"] + st["fp_singletons"]
    note("sampled parity: %d keys (%d present), %d Bloom bits" % (
        sample.size, int((want > 0).sum()), bits.size))
