"""Bloom filters of 2^30 to 2^36 bits per level on small inputs: the sizes of
the batched (2^35), served (up to 2^34) and 3 Gbp (2^36) workloads, whose
word and bit indices pass 2^32, checked exactly against the CPU oracle.  The
table and every statistic are compared whole; each level is compared at
every word the oracle sets, and the popcounts are equal, so no other bit is
set (kc_export_bloom_words reads the chosen words).

Every case prints its name and shape before touching the GPU.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import (STAT_MAP, assert_bloom_sparse, assert_same_table, note, oracle_params,
                      to_device, workload_chunks)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


CASES = [  # (name, m_log2, block_log2, h, n_counters, partitions_log2, table_slots)
    ("2^33 bits, 2^16-bit blocks", 33, 16, 4, 1, 0, 256),
    ("2^34 bits, 2^16-bit blocks, joint (served request shape)", 34, 16, 4, 2, 0, 128),
    ("2^35 bits, 2^18-bit blocks (batched shape)", 35, 18, 4, 1, 0, 512),
    ("2^36 bits, 2^16-bit blocks (3 Gbp shape)", 36, 16, 4, 1, 0, 64),
    ("2^36 bits, 2^19-bit blocks, 3 hashes", 36, 19, 3, 1, 17, 256),
    ("2^30 bits, 2^16-bit blocks, joint", 30, 16, 4, 2, 0, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_large_bloom_parity(case):
    name, m, bl, h, nc, plog, slots = case
    note("case: %s; 20000 reads of the 1 Mbp workload" % name)
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=20000)
    cfg = kc.Config(k=31, n_counters=nc, bloom_bits_log2=m, bloom_hashes=h, bloom_block_log2=bl,
                    seed=33 + m, partitions_log2=plog, table_slots=slots)
    half = 10000
    parts = [(b[:int(o[half])], o[:half + 1]),
             (b[int(o[half]):], o[half:] - o[half])] if nc == 2 else [(b, o)]
    with kc.KmerCounter(cfg) as c:
        for t, (pb, po) in enumerate(parts):
            db, do = to_device(pb, po)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        keys, counts = c.export()
        tags = np.repeat(np.arange(len(parts), dtype=np.uint8), [p[1].size - 1 for p in parts])
        ref = oracle.count(oracle_params(cfg), b, o, tags=tags if nc == 2 else None,
                           want_bloom="sparse")
        assert_bloom_sparse(c.export_bloom_words, ref, st)
    assert_same_table(keys, counts, ref.keys, ref.counts)
    for a, r in STAT_MAP.items():
        assert st[a] == ref.stats[r], (a, st[a], ref.stats[r])
    note("entries %d, F %d, touched words %d" % (st["entries"], st["fp_singletons"],
                                                ref.touched.size))


def test_served_request_at_2_34_bits():
    """A joint request of the served workload's shape (two counters, 2^34-bit
    levels of 2^16-bit blocks, 4 hashes) through the request server, beside a
    small one: both equal the oracle."""
    note("case: served joint request, 2^34 bits, 2^16-bit blocks, beside a 2^24-bit one")
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=16000)
    jobs = []
    for m, n in ((34, 16000), (24, 4000)):
        half = n // 2
        parts = [(b[:int(o[half])], o[:half + 1]),
                 (b[int(o[half]):int(o[n])], o[half:n + 1] - o[half])]
        cfg = kc.Config(k=31, n_counters=2, bloom_bits_log2=m, bloom_hashes=4,
                        bloom_block_log2=16, seed=m, table_slots=128)
        jobs.append((cfg, parts))
    with kc.Server(64 << 30, workers=2) as srv:
        dev = [[to_device(pb, po) for pb, po in parts] for _, parts in jobs]
        tickets = [srv.submit(cfg, d) for (cfg, _), d in zip(jobs, dev)]
        for (cfg, parts), t in zip(jobs, tickets):
            resp = srv.wait(t)
            assert resp.status == 0
            keys, counts = kc.response_table(resp, 2)
            st = resp.stats.as_dict()
            pb = np.concatenate([p[0] for p in parts])
            po = np.concatenate([parts[0][1], parts[1][1][1:] + parts[0][1][-1]])
            tags = np.repeat(np.arange(2, dtype=np.uint8), [p[1].size - 1 for p in parts])
            ref = oracle.count(oracle_params(cfg), pb, po, tags=tags, want_bloom="sparse")
            assert_bloom_sparse(lambda idx: kc.kc_export_bloom_words(ctypes.c_void_p(resp.ctx), idx),
                                ref, st)
            assert_same_table(keys, counts, ref.keys, ref.counts)
            for a, r in STAT_MAP.items():
                assert st[a] == ref.stats[r], (a, st[a], ref.stats[r])
            srv.release(t)
