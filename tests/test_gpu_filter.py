"""kc_filter_reads (paper Sec. II-B, Filter unit: the input is read again and
its k-mers looked up in the frequency table to select imbalanced ones)
against the oracle's lookup on the oracle's table, read by read: joint
counters at several thresholds, one-counter tables, ragged reads, keys in the
overflow table, and the error paths.

Every case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import note, oracle_params, pack_reads, random_reads, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def joint(seed, n=1500):
    normal = random_reads(seed, n, 40, 130, genome_len=3000)
    tumour = random_reads(seed + 1, n, 40, 130, genome_len=3000)
    return pack_reads(normal), pack_reads(tumour)


def oracle_table(cfg, chunks, counters):
    bases = np.concatenate([b for b, _ in chunks])
    offs, base, tags = [np.zeros(1, np.uint64)], 0, []
    for (b, o), t in zip(chunks, counters):
        offs.append(o[1:] + np.uint64(base))
        base += int(o[-1])
        tags.append(np.full(o.size - 1, t, np.uint8))
    return oracle.count(oracle_params(cfg), bases, np.concatenate(offs), tags=np.concatenate(tags),
                        want_bloom=False)


def gpu_filter(cfg, chunks, counters, probe, thresholds):
    """kc_filter_reads at each threshold pair, checked equal to
    kc_filter_reads_noalloc (which always probes keys, then counts; the
    allocating entry point reads keys marked with the selection when the
    windows outnumber half the table slots)."""
    import torch
    out = []
    with kc.KmerCounter(cfg) as c:
        for (b, o), t in zip(chunks, counters):
            db, do = to_device(b, o)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        pb, po = to_device(*probe)
        direct = torch.empty(max(1, po.numel() - 1), dtype=torch.int32, device="cuda")
        for tmin, nmax in thresholds:
            got = c.filter_reads(pb, po, tmin, nmax).cpu().numpy().view(np.uint32).copy()
            ref = c.filter_reads_noalloc(pb, po, tmin, nmax, direct)
            assert np.array_equal(got, ref.cpu().numpy().view(np.uint32)), (tmin, nmax)
            out.append(got)
    return st, out


THRESHOLDS = [(2, 0), (1, 1), (3, 2), (0, 0xFFFFFFFF), (1, 0xFFFFFFFF)]


@pytest.mark.parametrize("k,seed,slots", [(21, 81, 0), (27, 82, 0), (31, 83, 0), (31, 86, 128)])
def test_filter_joint_counters(k, seed, slots):
    note("case: filter, joint counters, k=%d, seed %d, table slots %s, tumour reads re-read"
         % (k, seed, slots or "auto"))
    normal, tumour = joint(seed)
    cfg = kc.Config(k=k, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=13,
                    partitions_log2=9, table_slots=slots, seed=seed)
    st, got = gpu_filter(cfg, [normal, tumour], [0, 1], tumour, THRESHOLDS)
    res = oracle_table(cfg, [normal, tumour], [0, 1])
    for (tmin, nmax), g in zip(THRESHOLDS, got):
        want = oracle.filter_reads(k, 2, res.keys, res.counts, tumour[0], tumour[1], tmin, nmax)
        assert np.array_equal(g, want), (tmin, nmax)
    assert got[0].any() and (got[0] < got[3]).any()


def test_filter_one_counter_ragged_reads_and_overflow():
    note("case: filter, one counter, 16 tables of 64 slots, ragged probe reads, seed 84")
    reads = random_reads(84, 2500, 30, 150, genome_len=3000)
    cfg = kc.Config(k=15, bloom_bits_log2=18, bloom_hashes=2, bloom_block_log2=14, partitions_log2=4,
                    table_slots=64, seed=84)
    probe_reads = ["", "ACG", "N" * 20] + random_reads(85, 400, 0, 97, genome_len=3000) + ["ACGTN" * 9]
    probe = pack_reads(probe_reads)
    th = [(2, 0), (5, 0), (1, 0)]
    st, got = gpu_filter(cfg, [pack_reads(reads)], [0], probe, th)
    assert st["overflow_keys"] > 0
    res = oracle_table(cfg, [pack_reads(reads)], [0])
    for (tmin, nmax), g in zip(th, got):
        want = oracle.filter_reads(15, 1, res.keys, res.counts, probe[0], probe[1], tmin, nmax)
        assert np.array_equal(g, want), (tmin, nmax)
    assert got[0][:3].tolist() == [0, 0, 0]


def test_filter_errors():
    import torch
    note("case: filter errors: before finalize, bad offsets, spilled tables, seed 86")
    normal, tumour = joint(86, n=600)
    cfg = kc.Config(k=25, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=14,
                    partitions_log2=8, table_slots=256, seed=86)
    with kc.KmerCounter(cfg) as c:
        db, do = to_device(*normal)
        c.insert_reads(db, do, counter=0)
        with pytest.raises(kc.KcError) as e:
            c.filter_reads(db, do, 1, 0)
        assert e.value.status == kc.KC_ERR_BAD_STATE
        c.finalize()
        bad = normal[1].copy()
        bad[-1] += 7  # ends past the bases
        with pytest.raises(kc.KcError) as e:
            c.filter_reads(db, torch.from_numpy(bad.view(np.int64)).cuda(), 1, 0)
        assert e.value.status == kc.KC_ERR_INVALID_ARG
        ok = c.filter_reads(db, do, 1, 0xFFFFFFFF)  # still usable afterwards
        assert ok.numel() == normal[1].size - 1
        c.spill(3)
        with pytest.raises(kc.KcError) as e:
            c.filter_reads(db, do, 1, 0)
        assert e.value.status == kc.KC_ERR_BAD_STATE
