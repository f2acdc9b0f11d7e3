"""The served workload at full size (512 timed joint tumour/normal requests
of 10^4-5·10^6 reads from the 300 Mbp normal and tumour samples, a 32 GB
budget, eight workers with at most 2^28 bases in flight, as bench.py serves
them).  Every request's statistics in the mix equal those of the same request
run alone (a one-worker server runs one job at a time), and for the 16
requests that tests/golden/make_digests.py counted with the CPU oracle (the
largest and 15 seeded ones) so does the whole output, in the mix and alone:
the sorted table (whole and per value range) and both Bloom levels.
"""
import ctypes
import os

import numpy as np
import pytest

import paper_1712_03254_amd as kc
from conftest import GOLDEN
from digest import STAT_KEYS, read_request_digests, table_digests, words_digest
from kc_cases import gpu_table_sorted, note

pytestmark = pytest.mark.gpu


def test_served_workload_mix_equals_alone_and_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth
    note("case: served_300mbp full size, 512 requests, 8 workers (cap 2^28 bases) against one")
    want = read_request_digests(os.path.join(GOLDEN, "digest_served_300mbp.txt"))
    w = synth.WORKLOADS["served_300mbp"]
    normal = w.make_genome(threads=16)
    tumour = w.make_tumour(normal)
    reads = [w.make_sample_reads(normal, 0, threads=16), w.make_sample_reads(tumour, 1, threads=16)]
    del normal, tumour
    L = w.lmax
    dev_b = [torch.from_numpy(b).cuda() for b, _ in reads]
    offs = torch.from_numpy(reads[0][1].view(np.int64)).cuda()
    del reads
    plan = w.request_plan()[w.warmup_requests:]
    jobs = []
    for n, s0, s1 in plan:
        n, s0, s1 = int(n), int(s0), int(s1)
        half = n // 2
        _, m, pl = w.request_params(n)
        cfg = kc.Config(k=w.k, n_counters=2, min_count=w.min_count, bloom_bits_log2=m,
                        bloom_hashes=w.bloom_hashes, bloom_block_log2=w.bloom_block_log2,
                        seed=w.seed, partitions_log2=pl)
        jobs.append((cfg, [(dev_b[0][s0 * L:(s0 + half) * L], offs[:half + 1]),
                           (dev_b[1][s1 * L:(s1 + half) * L], offs[:half + 1])]))
    for i, d in want.items():
        assert (d["reads"], d["normal"], d["tumour"]) == tuple(int(v) for v in plan[i])
        assert d["m"] == jobs[i][0].bloom_bits_log2

    def serve(workers, overlap):
        out = []
        with kc.Server(w.serve_budget, workers=workers, overlap_bases=overlap) as srv:
            tickets = [srv.submit(cfg, parts) for cfg, parts in jobs]
            for i, t in enumerate(tickets):
                r = srv.wait(t)
                assert r.status == kc.KC_OK, (i, r.status)
                st = r.stats.as_dict()
                rec = {"stats": {k: st[k] for k in STAT_KEYS}}
                if i in want:
                    keys, counts = kc.response_table(r, 2)
                    ks, cs = gpu_table_sorted(keys, counts)
                    rec["table"] = table_digests(ks, cs, w.k)
                    words = (1 << jobs[i][0].bloom_bits_log2) // 64
                    b1, b2 = kc.kc_export_bloom(ctypes.c_void_p(r.ctx), words)
                    rec["b1"], rec["b2"] = words_digest(b1), words_digest(b2)
                    del keys, counts, ks, cs, b1, b2
                out.append(rec)
                srv.release(t)
            u = srv.usage()
        note("%d worker(s): contexts created %d, evicted %d; cache %.1f GB"
             % (workers, u["created"], u["evicted"], u["cached_bytes"] / 1e9))
        return out

    mixed = serve(8, 1 << 28)
    alone = serve(1, 0)
    for i, (a, b) in enumerate(zip(mixed, alone)):
        assert a["stats"] == b["stats"], ("request", i, a["stats"], b["stats"])
    for i, d in want.items():
        for run in (mixed[i], alone[i]):
            assert run["stats"] == d["stats"], ("request", i, run["stats"], d["stats"])
            got = run["table"]
            for q, (g, r) in enumerate(zip(got["ranges"], d["ranges"])):
                assert tuple(g) == tuple(r), ("request", i, "value range", q)
            assert got["sha256"] == d["sha256"], ("request", i)
            assert run["b1"] == d["b1"] and run["b2"] == d["b2"], ("request", i)
    note("512 requests equal alone; %d equal the oracle's whole output" % len(want))
