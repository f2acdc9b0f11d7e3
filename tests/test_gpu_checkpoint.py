"""kc_checkpoint / kc_restore (paper Sec. II-B: checkpointable units dump
their Bloom filters and tables; Sec. III-D: swapped tables are found again
through metadata records in a reserved area): a restored context answers
exactly as the one that wrote the file - table, Bloom levels, statistics,
queries (resident and spilled partitions, overflow keys), stem items and the
filter - and the table equals the oracle's.  Corrupted files are rejected.

Every case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import (STAT_MAP, assert_same_table, note, oracle_params, pack_reads, random_reads,
                      to_device)

pytestmark = pytest.mark.gpu

SAME = ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount", "b2_popcount",
        "overflow_keys", "table_slots", "partitions_log2")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def snapshot(c, probe_keys, probe_reads=None):
    import torch
    keys, counts = c.export()
    b1, b2 = c.export_bloom()
    q = c.query(torch.from_numpy(probe_keys.view(np.int64)).cuda()).cpu().numpy().view(np.uint32)
    out = dict(keys=keys, counts=counts, b1=b1, b2=b2, q=q.copy(), stats=c.stats())
    stems, items = c.export_stems()
    order = np.argsort(stems.cpu().numpy().view(np.uint64), kind="stable")
    out["stems"] = stems.cpu().numpy().view(np.uint64)[order]
    out["items"] = items.cpu().numpy().view(np.uint16)[order]
    if probe_reads is not None:
        b, o = probe_reads
        out["filter"] = c.filter_reads(b, o, 2, 1).cpu().numpy().copy()
    return out


def assert_same(a, b):
    assert_same_table(a["keys"], a["counts"], b["keys"], b["counts"])
    assert np.array_equal(a["b1"], b["b1"]) and np.array_equal(a["b2"], b["b2"])
    assert np.array_equal(a["q"], b["q"])
    assert np.array_equal(a["stems"], b["stems"]) and np.array_equal(a["items"], b["items"])
    for k in SAME:
        assert a["stats"][k] == b["stats"][k], k
    if "filter" in a and "filter" in b:
        assert np.array_equal(a["filter"], b["filter"])


@pytest.mark.parametrize("tables,explicit,small", [(0, False, False), (0, True, False), (40, False, False),
                                                   (0, False, True)])
def test_checkpoint_round_trip(tmp_path, tables, explicit, small):
    note("case: checkpoint, budget %s tables, explicit spill %s, small tables %s, seed 91"
         % (tables or "all", explicit, small))
    normal = random_reads(91, 1500, 50, 120, genome_len=4000)
    tumour = random_reads(92, 1500, 50, 120, genome_len=4000)
    chunks = [pack_reads(normal), pack_reads(tumour)]
    cfg = kc.Config(k=25, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=14,
                    partitions_log2=4 if small else 8, table_slots=64 if small else 256, seed=91)
    if tables:
        cfg.hbm_table_budget_bytes = 256 * 16 * tables
    path = str(tmp_path / "count.kcckpt")
    rng = np.random.default_rng(91)
    with kc.KmerCounter(cfg) as c:
        for (b, o), t in zip(chunks, [0, 1]):
            db, do = to_device(b, o)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        if small:
            assert st["overflow_keys"] > 0
        keys, _ = c.export()
        probe = np.concatenate([keys, rng.integers(0, 1 << 50, 500, dtype=np.uint64)])
        tb, to = to_device(*chunks[1])
        before = snapshot(c, probe, None if tables else (tb, to))
        if explicit:
            c.spill(5)
            c.spill(200)
            before_q = snapshot(c, probe)
            assert np.array_equal(before_q["q"], before["q"])
        c.checkpoint(path)
    with kc.KmerCounter.restore(path) as r:
        after = snapshot(r, probe, None if tables else (tb, to))
        st2 = r.stats()
        assert st2["spilled_partitions"] == (256 - tables if tables else 0)
    assert_same(before, after)
    # and the restored table is the oracle's
    bases = np.concatenate([chunks[0][0], chunks[1][0]])
    o0, o1 = chunks[0][1], chunks[1][1]
    offs = np.concatenate([o0, o1[1:] + o0[-1]])
    tags = np.concatenate([np.zeros(o0.size - 1, np.uint8), np.ones(o1.size - 1, np.uint8)])
    ref = oracle.count(oracle_params(cfg), bases, offs, tags=tags)
    assert_same_table(after["keys"], after["counts"], ref.keys, ref.counts)
    for a, b in STAT_MAP.items():
        assert after["stats"][a] == ref.stats[b]


def test_restored_context_counts_again_and_bad_files(tmp_path):
    import ctypes
    note("case: restored context reset and reused; corrupted checkpoints, seed 93")
    reads = random_reads(93, 1200, 40, 110, genome_len=3000)
    cfg = kc.Config(k=21, bloom_bits_log2=18, bloom_hashes=3, bloom_block_log2=12, seed=93)
    path = str(tmp_path / "one.kcckpt")
    b, o = pack_reads(reads)
    db, do = to_device(b, o)
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        c.finalize()
        c.checkpoint(path)
        want_keys, want_counts = c.export()
    with kc.KmerCounter.restore(path) as r:
        r.reset()
        r.insert_reads(db, do)
        r.finalize()
        keys, counts = r.export()
        assert_same_table(keys, counts, want_keys, want_counts)
    raw = open(path, "rb").read()
    lib = kc.load()
    h = ctypes.c_void_p()
    cut = tmp_path / "cut.kcckpt"
    cut.write_bytes(raw[: len(raw) - 100])
    assert lib.kc_restore(str(cut).encode(), 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    assert not h.value
    with pytest.raises(kc.KcError):
        kc.kc_checkpoint(None, path)  # no context
