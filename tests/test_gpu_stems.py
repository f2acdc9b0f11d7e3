"""kc_export_stems (paper Sec. II-A stems, Sec. III-D items of 16 normal and
16 tumour counts per stem) against the oracle's stem items of the oracle's
final table, element by element after sorting by stem: resident tables, the
overflow table, spilled tables, joint counters, palindromic stems (even k),
many k-mers per stem (small k) and counts past 16 bits.

Every case prints its name, seed and shape before touching the GPU.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import note, oracle_params, pack_reads, random_reads, to_device, workload_chunks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def gpu_stems(cfg, chunks, counters=None):
    counters = counters or [0] * len(chunks)
    with kc.KmerCounter(cfg) as c:
        for (b, o), t in zip(chunks, counters):
            db, do = to_device(b, o)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        stems, counts = c.export_stems()
        stems = stems.cpu().numpy().view(np.uint64)
        counts = counts.cpu().numpy().view(np.uint16)
    return st, stems, counts


def oracle_stems(cfg, chunks, counters=None):
    bases = np.concatenate([b for b, _ in chunks])
    offs, base, tags = [np.zeros(1, np.uint64)], 0, []
    for i, (b, o) in enumerate(chunks):
        offs.append(o[1:] + np.uint64(base))
        base += int(o[-1])
        tags.append(np.full(o.size - 1, (counters or [0] * len(chunks))[i], np.uint8))
    res = oracle.count(oracle_params(cfg), bases, np.concatenate(offs), tags=np.concatenate(tags),
                       want_bloom=False)
    return res, oracle.stem_items(cfg.k, cfg.n_counters, res.keys, res.counts)


def assert_same_items(got, want):
    stems, counts = got
    ws, wc = want
    order = np.argsort(stems, kind="stable")
    assert np.array_equal(stems[order], ws)
    assert np.array_equal(counts[order], wc)


def test_stems_plain_1mbp_slice():
    note("case: stems, plain_1mbp first 8000 reads, k=31")
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=8000)
    cfg = kc.Config(k=31, bloom_bits_log2=22, bloom_hashes=3, bloom_block_log2=14, seed=1)
    st, stems, counts = gpu_stems(cfg, [(b, o)])
    res, want = oracle_stems(cfg, [(b, o)])
    assert stems.size <= st["entries"] == res.keys.size
    assert_same_items((stems, counts), want)
    note("%d table entries -> %d stem items" % (st["entries"], stems.size))


@pytest.mark.parametrize("k,seed", [(5, 41), (8, 42), (20, 43), (24, 44)])
def test_stems_joint_counters_and_small_or_even_k(k, seed):
    note("case: stems, joint counters, k=%d, seed %d" % (k, seed))
    normal = random_reads(seed, 1500, 40, 120, genome_len=3000)
    tumour = random_reads(seed + 100, 1500, 40, 120, genome_len=3000)
    chunks = [pack_reads(normal), pack_reads(tumour)]
    cfg = kc.Config(k=k, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=12,
                    partitions_log2=9, seed=seed)
    st, stems, counts = gpu_stems(cfg, chunks, counters=[0, 1])
    res, want = oracle_stems(cfg, chunks, counters=[0, 1])
    assert_same_items((stems, counts), want)
    assert counts[:, 1].any()  # the tumour half is filled


def test_stems_overflow_and_saturation():
    note("case: stems, 64-slot tables (overflow table), a k-mer seen 70000 times, k=9")
    reads = random_reads(51, 2000, 60, 140, genome_len=4000) + ["A" * 70008]
    # 16 partitions of 64 slots: far fewer slots than passing keys
    cfg = kc.Config(k=9, bloom_bits_log2=18, bloom_hashes=2, bloom_block_log2=14, partitions_log2=4,
                    table_slots=64, seed=51)
    chunks = [pack_reads(reads)]
    st, stems, counts = gpu_stems(cfg, chunks)
    assert st["overflow_keys"] > 0
    res, want = oracle_stems(cfg, chunks)
    assert_same_items((stems, counts), want)
    assert int(counts.max()) == 65535  # AAAAAAAAA: 70000 occurrences, saturated


@pytest.mark.parametrize("tables", [1, 100])
def test_stems_with_spilled_tables(tables):
    note("case: stems, table budget of %d tables of 256 (spilled partitions staged back)" % tables)
    reads = random_reads(61, 3000, 50, 120, genome_len=6000)
    cfg = kc.Config(k=27, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=14,
                    partitions_log2=8, table_slots=256, seed=61)
    cfg.hbm_table_budget_bytes = 256 * 16 * tables
    chunks = [pack_reads(reads[:1500]), pack_reads(reads[1500:])]
    st, stems, counts = gpu_stems(cfg, chunks, counters=[0, 1])
    assert st["spilled_partitions"] == 256 - tables
    res, want = oracle_stems(cfg, chunks, counters=[0, 1])
    assert_same_items((stems, counts), want)


def test_stems_capacity_and_state_errors():
    import torch
    note("case: stems, capacity below the item count; before finalize; k=2")
    reads = random_reads(71, 500, 60, 100, genome_len=2000)
    cfg = kc.Config(k=21, bloom_bits_log2=18, bloom_hashes=3, bloom_block_log2=12, seed=71)
    b, o = pack_reads(reads)
    db, do = to_device(b, o)
    lib = kc.load()
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        n = ctypes.c_uint64(0)
        assert lib.kc_export_stems(c.ctx, None, None, 0, ctypes.byref(n), None) == kc.KC_ERR_BAD_STATE
        c.finalize()
        stems = torch.empty(4, dtype=torch.int64, device="cuda")
        counts = torch.empty((4, 32), dtype=torch.int16, device="cuda")
        rc = lib.kc_export_stems(c.ctx, stems.data_ptr(), counts.data_ptr(), 4, ctypes.byref(n), None)
        assert rc == kc.KC_ERR_INVALID_ARG and n.value > 4
        full, _ = c.export_stems()
        assert full.numel() == n.value
    with kc.KmerCounter(kc.Config(k=2, bloom_bits_log2=12, bloom_hashes=2, bloom_block_log2=8)) as c:
        c.insert_reads(db, do)
        c.finalize()
        with pytest.raises(kc.KcError):
            c.export_stems()
