"""Writes the whole-output digest of a workload from the CPU oracle.

    python tests/golden/make_digests.py plain_100mbp [--threads N]

Calls only the oracle (``oracle.count_ranges``: value-range passes over
every window) and the seeded input generator (``synth``); nothing here runs
the GPU library.  The result, ``tests/golden/digest_<workload>.txt``, holds
every statistic, the SHA-256 of the sorted table (whole and per value range)
and of both Bloom levels; ``tests/test_gpu_full.py`` digests the library's
output at the same workload and compares.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402
from digest import (TableDigest, served_subset, table_digests, words_digest,  # noqa: E402
                    write_digest_file, write_request_digests)

STATS = {"n_valid": "n_valid", "n_pass": "n_pass", "entries": "entries",
         "sum_counts": "sum_counts", "fp_singletons": "fp_singletons",
         "b1_popcount": "b1_pop", "b2_popcount": "b2_pop"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--qbits", type=int, default=0)
    ap.add_argument("--stream", action="store_true",
                    help="digest each value range's table as its pass ends and screen in a second "
                         "sweep (for workloads whose table and singletons do not fit in memory)")
    args = ap.parse_args()
    w = synth.WORKLOADS[args.workload]
    if w.requests:
        served(w, args)
        return
    t0 = time.time()
    genome = w.make_genome()
    # a batched workload's chunks are consecutive reads of one read stream
    # (Workload.make_chunk), so all of them together are its first n reads
    n_reads = int(w.chunk_plan().sum()) if w.batch_chunks else w.n_reads
    bases, offsets = w.make_reads(genome, first=0, n=n_reads)
    del genome
    p = oracle.Params(k=w.k, n_counters=w.n_counters, min_count=w.min_count,
                      m_log2=w.bloom_bits_log2, h=w.bloom_hashes,
                      block_log2=min(w.bloom_block_log2, w.bloom_bits_log2), seed=w.seed)
    t1 = time.time()
    if args.stream:
        if args.qbits < 4:
            raise SystemExit("--stream needs --qbits 4 or more (each range inside one digest range)")
        td = TableDigest(w.k)
        res = oracle.count_ranges(p, bases, offsets, threads=args.threads, qbits=args.qbits,
                                  keep_singles=False, on_range=lambda q, k, c: td.update(k, c))
        table = td.result()
    else:
        res = oracle.count_ranges(p, bases, offsets, threads=args.threads, qbits=args.qbits)
        table = table_digests(res.keys, res.counts, w.k)
    t2 = time.time()
    stats = {k: res.stats[v] for k, v in STATS.items()}
    b1, b2 = words_digest(res.b1), words_digest(res.b2)
    out = os.path.join(HERE, "digest_%s.txt" % w.name)
    header = [
        "Whole output of the CPU oracle (value-range passes) at workload %s:" % w.name,
        "genome %d bp, %d reads of %d-%d bp%s, substitutions %g, N rate %g, seed %d;"
        % (w.genome_len, n_reads, w.lmin, w.lmax,
           " in %d chunks" % w.batch_chunks if w.batch_chunks else "", w.err, w.nrate, w.seed),
        "k=%d, %d counter(s), min_count %d, Bloom 2^%d bits per level, %d hashes, blocks of 2^%d bits."
        % (w.k, w.n_counters, w.min_count, w.bloom_bits_log2, w.bloom_hashes,
           min(w.bloom_block_log2, w.bloom_bits_log2)),
        "Written by: python tests/golden/make_digests.py %s%s%s (oracle %.0f s, input %.0f s)."
        % (w.name, "".join(" --%s %d" % (k, v) for k, v in (("threads", args.threads),
                                                           ("qbits", args.qbits)) if v),
           " --stream" if args.stream else "", t2 - t1, t1 - t0),
        "Table stream: entries ascending by key, key <u8 then counts <u4; ranges by the top 4",
        "bits of the 2k-bit code: 'range q entries sum_of_counts sha256'.",
    ]
    write_digest_file(out, header, stats, table, b1, b2)
    print("wrote %s in %.0f s" % (out, time.time() - t0))


def served(w, args):
    """A served workload: the whole output of each request of a seeded subset
    (digest.served_subset of the timed requests: the largest and 15 others),
    each request counted alone by the oracle with its own Bloom size
    (Workload.request_params) and two counters, its normal reads in counter 0
    and its tumour reads in counter 1."""
    t0 = time.time()
    normal = w.make_genome()
    tumour = w.make_tumour(normal)
    samples = [w.make_sample_reads(normal, 0), w.make_sample_reads(tumour, 1)]
    del normal, tumour
    plan = w.request_plan()[w.warmup_requests:]
    pick = served_subset(plan[:, 0], seed=w.seed)
    L = w.lmax
    t1 = time.time()
    records = []
    for i in pick:
        n, s0, s1 = (int(v) for v in plan[i])
        half = n // 2
        _, m, _ = w.request_params(n)
        bases = np.concatenate([samples[0][0][s0 * L:(s0 + half) * L],
                                samples[1][0][s1 * L:(s1 + half) * L]])
        offsets = np.arange(2 * half + 1, dtype=np.uint64) * np.uint64(L)
        tags = np.repeat(np.array([0, 1], np.uint8), half)
        p = oracle.Params(k=w.k, n_counters=2, min_count=w.min_count, m_log2=m, h=w.bloom_hashes,
                          block_log2=min(w.bloom_block_log2, m), seed=w.seed)
        res = oracle.count_ranges(p, bases, offsets, tags=tags, threads=args.threads,
                                  qbits=args.qbits)
        records.append({"index": i, "reads": n, "normal": s0, "tumour": s1, "m": m,
                        "stats": {k: res.stats[v] for k, v in STATS.items()},
                        "table": table_digests(res.keys, res.counts, w.k),
                        "b1": words_digest(res.b1), "b2": words_digest(res.b2)})
        print("request %d: %d reads, m %d, %d entries" % (i, n, m, res.stats["entries"]),
              flush=True)
        del res, bases
    t2 = time.time()
    out = os.path.join(HERE, "digest_%s.txt" % w.name)
    header = [
        "Whole output of the CPU oracle (value-range passes) for a subset of the timed requests of",
        "workload %s: the largest and 15 drawn with seed %d (digest.served_subset), each counted" % (
            w.name, w.seed),
        "alone: its normal reads (reads normal .. normal+n/2-1 of sample 0) in counter 0, its tumour",
        "reads (tumour .. tumour+n/2-1 of sample 1) in counter 1; k=%d, min_count %d, Bloom 2^m bits"
        % (w.k, w.min_count),
        "per level (m per request), %d hashes, blocks of 2^%d bits; request i is timed request i."
        % (w.bloom_hashes, w.bloom_block_log2),
        "Written by: python tests/golden/make_digests.py %s%s (oracle %.0f s, input %.0f s)."
        % (w.name, "".join(" --%s %d" % (k, v) for k, v in (("threads", args.threads),
                                                           ("qbits", args.qbits)) if v),
           t2 - t1, t1 - t0),
        "Table stream per request: entries ascending by key, key <u8 then counts <u4 (normal,",
        "tumour); ranges by the top 4 bits of the 2k-bit code.",
    ]
    write_request_digests(out, header, records)
    print("wrote %s in %.0f s" % (out, time.time() - t0))


if __name__ == "__main__":
    main()
