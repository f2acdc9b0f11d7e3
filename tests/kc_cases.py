"""Shared helpers of the GPU tests: seeded inputs, device upload, comparisons.

Test infrastructure; the product library never imports it.
"""
from __future__ import annotations

import random
import sys

import numpy as np

import oracle
import paper_1712_03254_amd as kc
import synth


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def pack_reads(reads):
    offs = np.zeros(len(reads) + 1, dtype=np.uint64)
    for i, r in enumerate(reads):
        offs[i + 1] = offs[i] + len(r)
    data = "".join(reads).encode()
    bases = np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(0, np.uint8)
    return bases, offs


def random_reads(seed, n, lmin, lmax, genome_len=2000, err=0.02, nfrac=0.01, junk="NnRX."):
    """Reads sampled from a short random genome (so k-mers repeat), both strands,
    with substitutions and invalid bytes."""
    rng = random.Random(seed)
    genome = "".join(rng.choice("ACGT") for _ in range(genome_len))
    comp = str.maketrans("ACGT", "TGCA")
    out = []
    for _ in range(n):
        L = rng.randint(lmin, lmax)
        L = min(L, genome_len)
        st = rng.randint(0, genome_len - L)
        s = list(genome[st:st + L])
        for j in range(L):
            u = rng.random()
            if u < err:
                s[j] = rng.choice("ACGT")
            elif u < err + nfrac:
                s[j] = rng.choice(junk)
        r = "".join(s)
        if rng.random() < 0.5:
            r = r[::-1].translate(comp)
        out.append(r)
    return out


def to_device(bases, offsets):
    import torch
    b = torch.from_numpy(np.ascontiguousarray(bases)).to("cuda")
    o = torch.from_numpy(np.ascontiguousarray(offsets).view(np.int64)).to("cuda")
    return b, o


def oracle_params(cfg: kc.Config) -> oracle.Params:
    return oracle.Params(k=cfg.k, n_counters=cfg.n_counters, min_count=cfg.min_count,
                         m_log2=cfg.bloom_bits_log2, h=cfg.bloom_hashes,
                         block_log2=min(cfg.bloom_block_log2, cfg.bloom_bits_log2),
                         seed=cfg.seed)


def run_gpu(cfg: kc.Config, chunks, counters=None, want_bloom=True):
    """chunks: list of (bases, offsets) numpy pairs, inserted one call each."""
    import torch
    counters = counters or [0] * len(chunks)
    with kc.KmerCounter(cfg) as c:
        for (b, o), t in zip(chunks, counters):
            db, do = to_device(b, o)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        torch.cuda.synchronize()
        keys, counts = c.export()
        b1 = b2 = None
        if want_bloom:
            b1, b2 = c.export_bloom()
        return dict(keys=keys, counts=counts, b1=b1, b2=b2, stats=st)


def sorted_table(keys, counts):
    order = np.argsort(keys, kind="stable")
    return keys[order], counts[order]


def assert_same_table(got_keys, got_counts, want_keys, want_counts):
    gk, gc = sorted_table(np.asarray(got_keys), np.asarray(got_counts))
    wk, wc = sorted_table(np.asarray(want_keys), np.asarray(want_counts))
    assert gk.shape == wk.shape, (gk.shape, wk.shape)
    assert np.array_equal(gk, wk)
    assert np.array_equal(gc, wc)


STAT_MAP = {"n_valid": "n_valid", "n_pass": "n_pass", "entries": "entries",
            "sum_counts": "sum_counts", "fp_singletons": "fp_singletons",
            "b1_popcount": "b1_pop", "b2_popcount": "b2_pop"}


def assert_parity(cfg: kc.Config, chunks, counters=None):
    """Full element-wise parity of table, Bloom levels and statistics."""
    g = run_gpu(cfg, chunks, counters)
    bases = np.concatenate([c[0] for c in chunks]) if chunks else np.zeros(0, np.uint8)
    offs = [np.zeros(1, np.uint64)]
    base = 0
    tags = []
    for (b, o), t in zip(chunks, counters or [0] * len(chunks)):
        offs.append(o[1:] + np.uint64(base))
        base += int(o[-1])
        tags += [t] * (o.size - 1)
    offs = np.concatenate(offs)
    ref = oracle.count(oracle_params(cfg), bases, offs,
                       tags=np.array(tags, np.uint8) if cfg.n_counters > 1 else None)
    assert_same_table(g["keys"], g["counts"], ref.keys, ref.counts)
    assert np.array_equal(g["b1"], ref.b1)
    assert np.array_equal(g["b2"], ref.b2)
    for a, b in STAT_MAP.items():
        assert g["stats"][a] == ref.stats[b], (a, g["stats"][a], ref.stats[b])
    assert g["stats"]["passed_distinct"] == ref.stats["entries"] + ref.stats["fp_singletons"] or \
        cfg.min_count > 2
    return g, ref


def workload_chunks(name, n_reads=None, first=0):
    w = synth.WORKLOADS[name]
    genome = w.make_genome()
    n = w.n_reads if n_reads is None else n_reads
    b, o = w.make_reads(genome, first=first, n=n)
    return w, genome, b, o


def workload_config(w: synth.Workload, **over) -> kc.Config:
    cfg = kc.Config(k=w.k, n_counters=w.n_counters, min_count=w.min_count,
                    bloom_bits_log2=w.bloom_bits_log2, bloom_hashes=w.bloom_hashes,
                    bloom_block_log2=w.bloom_block_log2, seed=w.seed,
                    partitions_log2=w.partitions_log2,
                    hbm_table_budget_bytes=w.table_budget)
    for k_, v in over.items():
        setattr(cfg, k_, v)
    return cfg


def gpu_table_sorted(keys, counts):
    """The exported table sorted by key on the device (the table can hold 10^8
    entries and more); returns host arrays."""
    import torch
    k = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).cuda()
    order = torch.argsort(k)  # keys < 2^62: signed order is unsigned order
    ks = k[order].cpu().numpy().view(np.uint64)
    c = torch.from_numpy(np.ascontiguousarray(counts).view(np.int32)).cuda()
    cs = c[order].cpu().numpy().view(np.uint32)
    return ks, cs


def assert_bloom_sparse(counter_words, ref, stats):
    """Both Bloom levels equal the oracle's, from its nonzero words: the
    library's words at those indices are the oracle's and its popcounts are
    the oracle's, so no bit is set anywhere else."""
    g1, g2 = counter_words(ref.touched)
    assert np.array_equal(g1, ref.t1)
    assert np.array_equal(g2, ref.t2)
    pop = lambda v: int(np.unpackbits(np.ascontiguousarray(v).view(np.uint8)).sum())
    assert stats["b1_popcount"] == ref.stats["b1_pop"] == pop(ref.t1)
    assert stats["b2_popcount"] == ref.stats["b2_pop"] == pop(ref.t2)
