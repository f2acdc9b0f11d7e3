"""kc_filter_reads_noalloc, the allocation-free variant of kc_filter_reads
for callers that cannot allocate device memory: through the C ABI, its
per-read counts equal kc_filter_reads' on two calls in a row (the second
with a smaller, ragged input, so stale scratch from the first call would
show), and the oracle's on the second; a batch past the scratch size is
rejected on the host.

Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import note, pack_reads, random_reads, to_device, workload_chunks

pytestmark = pytest.mark.gpu


def test_noalloc_filter_equals_filter_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: joint table of 16000 reads (1 Mbp workload); noalloc filter vs filter, "
         "20000 reads then 700 ragged reads")
    w, _, b, o = workload_chunks("plain_1mbp")
    cfg = kc.Config(k=w.k, n_counters=2, bloom_bits_log2=w.bloom_bits_log2,
                    bloom_hashes=w.bloom_hashes, bloom_block_log2=w.bloom_block_log2, seed=w.seed,
                    partitions_log2=w.partitions_log2)
    half = 8000
    parts = [(b[:int(o[half])], o[:half + 1]),
             (b[int(o[half]):int(o[2 * half])], o[half:2 * half + 1] - o[half])]
    small = pack_reads(random_reads(515, 700, 0, 250, genome_len=1_000_000, nfrac=0.005))
    with kc.KmerCounter(cfg) as c:
        for t, (pb, po) in enumerate(parts):
            db, do = to_device(pb, po)
            c.insert_reads(db, do, counter=t)
        c.finalize()
        keys, counts = c.export()
        for name, (rb, ro) in (("all 20000 reads", (b, o)), ("700 ragged reads", small)):
            note("call: %s (%d bases)" % (name, rb.size))
            db, do = to_device(rb, ro)
            n = ro.size - 1
            for tmin, nmax in ((1, 0), (2, 3), (0, 0xFFFFFFFF)):
                want = c.filter_reads(db, do, tmin, nmax).cpu().numpy()
                out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
                got = c.filter_reads_noalloc(db, do, tmin, nmax, out).cpu().numpy()
                assert np.array_equal(got, want), (name, tmin, nmax)
        # the second (small) batch against the oracle's lookup of the oracle's view
        # of the exported table
        db, do = to_device(*small)
        out = torch.full((small[1].size - 1,), -1, dtype=torch.int32, device="cuda")
        got = c.filter_reads_noalloc(db, do, 2, 3, out).cpu().numpy().view(np.uint32)
        order = np.argsort(keys)
        ref = oracle.filter_reads(cfg.k, 2, keys[order], counts[order], small[0], small[1], 2, 3)
        assert np.array_equal(got, ref)


def test_noalloc_filter_rejects_batches_past_its_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note("case: noalloc filter, batch of 2^25 + 1 bases (host-side rejection)")
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=2000)
    cfg = kc.Config(k=w.k, bloom_bits_log2=w.bloom_bits_log2, bloom_hashes=w.bloom_hashes,
                    bloom_block_log2=w.bloom_block_log2, seed=w.seed)
    with kc.KmerCounter(cfg) as c:
        db, do = to_device(b, o)
        c.insert_reads(db, do)
        c.finalize()
        n = (1 << 25) + 1
        big = torch.full((n,), ord("A"), dtype=torch.uint8, device="cuda")
        offs = torch.tensor([0, n], dtype=torch.int64, device="cuda")
        out = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(kc.KcError) as e:
            c.filter_reads_noalloc(big, offs, 1, 0, out)
        assert e.value.status == kc.KC_ERR_INVALID_ARG
        # the context still works afterwards
        got = c.filter_reads_noalloc(db, do, 0, 0xFFFFFFFF, torch.zeros(o.size - 1, dtype=torch.int32,
                                                                         device="cuda"))
        assert int(got.to(torch.int64).sum().item()) == c.stats()["n_valid"]
