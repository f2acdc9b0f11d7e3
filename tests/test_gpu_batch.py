"""Batched form (kc_count_batch, one hipGraph launch per batch) against the
CPU oracle, element by element, through the C ABI; graph replays against the
first run; the autotuner's choice against the default configuration.

Every case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import (STAT_MAP, assert_same_table, note, oracle_params, pack_reads, random_reads,
                      to_device)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def ragged_chunks(seed, n_chunks, genome_len=5000):
    """Chunks of uneven size: some empty, some of one read, some with empty
    reads, totals not multiples of 32."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_chunks):
        kind = i % 7
        if kind == 0:
            reads = []
        elif kind == 1:
            reads = random_reads(seed * 100 + i, 1, 40, 90, genome_len=genome_len)
        elif kind == 2:
            reads = ["", "ACGT", ""] + random_reads(seed * 100 + i, 30, 0, 140, genome_len=genome_len)
        else:
            n = int(rng.integers(50, 600))
            reads = random_reads(seed * 100 + i, n, 20, 170, genome_len=genome_len)
        out.append(pack_reads(reads))
    return out


def oracle_of(cfg, chunks, tags=None):
    bases = np.concatenate([c[0] for c in chunks]) if chunks else np.zeros(0, np.uint8)
    offs = [np.zeros(1, np.uint64)]
    base = 0
    for b, o in chunks:
        offs.append(o[1:] + np.uint64(base))
        base += int(o[-1])
    return oracle.count(oracle_params(cfg), bases, np.concatenate(offs), tags=tags)


def run_batch(c, dev_chunks, counter=0):
    import torch
    st = c.count_batch(dev_chunks, counter=counter)
    torch.cuda.synchronize()
    keys, counts = c.export()
    b1, b2 = c.export_bloom()
    return dict(keys=keys, counts=counts, b1=b1, b2=b2, stats=st)


def assert_matches_oracle(g, ref):
    assert_same_table(g["keys"], g["counts"], ref.keys, ref.counts)
    assert np.array_equal(g["b1"], ref.b1)
    assert np.array_equal(g["b2"], ref.b2)
    for a, b in STAT_MAP.items():
        assert g["stats"][a] == ref.stats[b], (a, g["stats"][a], ref.stats[b])


@pytest.mark.parametrize("group_log2", [0, 17, 18])
def test_batch_parity(group_log2):
    note("case: batch of 40 ragged chunks, group_bases_log2=%d, seed 61" % group_log2)
    chunks = ragged_chunks(61, 40)
    cfg = kc.Config(k=25, bloom_bits_log2=22, bloom_hashes=4, bloom_block_log2=14,
                    partitions_log2=10, seed=61, group_bases_log2=group_log2)
    ref = oracle_of(cfg, chunks)
    dev = [to_device(b, o) for b, o in chunks]
    with kc.KmerCounter(cfg) as c:
        g = run_batch(c, dev)
        assert_matches_oracle(g, ref)
        if group_log2 == 17:  # the largest chunk (< 2^17 bases) fits one segment
            assert g["stats"]["n_segments"] > 4
        # queries on the batch's tables
        import torch
        q = torch.from_numpy(ref.keys.view(np.int64)).cuda()
        out = c.query(q).cpu().numpy().astype(np.uint32)
        assert np.array_equal(out, ref.counts)


def test_batch_overflow_table_fill_falls_back_to_the_eager_path():
    """Tables of 64 slots against ~1.1·10^5 passing keys: the overflow table the
    graph was built with fills, so the call counts again on the eager path,
    which grows the table; the result equals the oracle's, and a second batch
    on the same context does the same."""
    note("case: batch of 8 chunks x 2000 reads x 100 bp from a 2e5 bp genome, 256 tables of "
         "64 slots (overflow fill in the graph), seed 67")
    chunks = [pack_reads(random_reads(6700 + i, 2000, 100, 100, genome_len=200000))
              for i in range(8)]
    cfg = kc.Config(k=31, bloom_bits_log2=22, bloom_hashes=4, bloom_block_log2=14,
                    partitions_log2=8, table_slots=64, seed=67)
    ref = oracle_of(cfg, chunks)
    dev = [to_device(b, o) for b, o in chunks]
    with kc.KmerCounter(cfg) as c:
        for rep in range(2):
            g = run_batch(c, dev)
            st = g["stats"]
            note("rep %d: overflow keys %d, retries %d" % (rep, st["overflow_keys"], st["retries"]))
            assert st["overflow_keys"] > 50_000
            assert st["retries"] >= 1
            assert_matches_oracle(g, ref)
            c.reset()


def test_batch_graph_replays_with_eager_work_between():
    """The captured graph is replayed after kc_reset; between replays the
    program runs its own eager work (another context's plain count, torch
    ops, synchronisations); every replay equals the first run and the oracle."""
    import torch
    note("case: batch graph replayed 4 times, seed 62")
    chunks = ragged_chunks(62, 25)
    cfg = kc.Config(k=21, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=12,
                    partitions_log2=9, seed=62, group_bases_log2=17)
    ref = oracle_of(cfg, chunks)
    dev = [to_device(b, o) for b, o in chunks]
    other_cfg = kc.Config(k=19, bloom_bits_log2=18, bloom_hashes=2, bloom_block_log2=10, seed=9)
    with kc.KmerCounter(cfg) as c, kc.KmerCounter(other_cfg) as other:
        first = run_batch(c, dev)
        assert_matches_oracle(first, ref)
        for rep in range(3):
            other.reset()
            b, o = to_device(*chunks[3 + rep])
            other.insert_reads(b, o)
            other.finalize()
            x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
            assert int((x * 3).sum().item()) == 3 * ((1 << 20) - 1) * (1 << 20) // 2
            torch.cuda.synchronize()
            c.reset()
            g = run_batch(c, dev)
            assert_same_table(g["keys"], g["counts"], first["keys"], first["counts"])
            assert np.array_equal(g["b1"], first["b1"]) and np.array_equal(g["b2"], first["b2"])
            for k in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons"):
                assert g["stats"][k] == first["stats"][k]
            assert g["stats"]["kernel_launches"]["graph"] == 1


def test_batch_then_plain_on_same_context():
    """An eager insert after a batch drops the graph (its buffers may move);
    the next batch captures a new one.  All three results match the oracle."""
    note("case: batch, plain, batch on one context, seed 63")
    chunks = ragged_chunks(63, 12)
    cfg = kc.Config(k=23, bloom_bits_log2=20, bloom_hashes=4, bloom_block_log2=12, seed=63)
    ref = oracle_of(cfg, chunks)
    dev = [to_device(b, o) for b, o in chunks]
    with kc.KmerCounter(cfg) as c:
        assert_matches_oracle(run_batch(c, dev), ref)
        c.reset()
        for b, o in dev:
            c.insert_reads(b, o)
        c.finalize()
        keys, counts = c.export()
        assert_same_table(keys, counts, ref.keys, ref.counts)
        c.reset()
        assert_matches_oracle(run_batch(c, dev), ref)


def test_batch_two_counters_and_errors():
    import torch
    note("case: batch into counter 1 of a joint table; bad offsets; budget; seed 64")
    chunks = ragged_chunks(64, 9)
    cfg = kc.Config(k=27, n_counters=2, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=12,
                    seed=64)
    bases = np.concatenate([c[0] for c in chunks])
    nreads = sum(c[1].size - 1 for c in chunks)
    ref = oracle_of(cfg, chunks, tags=np.ones(nreads, np.uint8))
    dev = [to_device(b, o) for b, o in chunks]
    with kc.KmerCounter(cfg) as c:
        g = run_batch(c, dev, counter=1)
        assert_matches_oracle(g, ref)
        assert int(g["counts"][:, 0].sum()) == 0
        c.reset()
        bad = list(dev)
        b, o = chunks[4]
        o_bad = o.copy()
        o_bad[-1] += 1
        bad[4] = (dev[4][0], torch.from_numpy(o_bad.view(np.int64)).cuda())
        with pytest.raises(kc.KcError) as e:
            c.count_batch(bad)
        assert e.value.status == kc.KC_ERR_INVALID_ARG
        assert_matches_oracle(run_batch(c, dev, counter=1), ref)
    del bases
    small = kc.Config(k=27, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=12, seed=64,
                      hbm_table_budget_bytes=1 << 20)
    with kc.KmerCounter(small) as c:
        with pytest.raises(kc.KcError) as e:
            c.count_batch(dev)
        assert e.value.status == kc.KC_ERR_OVER_BUDGET


def test_autotune_choice_is_result_neutral():
    note("case: autotuner over a 30-chunk batch, seed 65")
    chunks = ragged_chunks(65, 30, genome_len=20000)
    cfg = kc.Config(k=31, bloom_bits_log2=22, bloom_hashes=4, bloom_block_log2=14, seed=65)
    ref = oracle_of(cfg, chunks)
    dev = [to_device(b, o) for b, o in chunks]
    best, trials = kc.autotune_batch(cfg, dev)
    note("trials: %s" % [(t["partitions_log2"], t["table_slots"], t["scatter_bits"],
                          t["shuffle_tile_log2"], round(t["ms"], 3), t["status"]) for t in trials])
    assert len(trials) >= 6  # the start and its neighbours along each dimension
    assert {t["shuffle_tile_log2"] for t in trials} >= {12, 13}  # the tile size is searched
    assert all(t["status"] == 0 for t in trials)
    fastest = min(t["ms"] for t in trials)
    assert any(t["ms"] == fastest and t["partitions_log2"] == best.partitions_log2 and
               t["table_slots"] == best.table_slots for t in trials)
    for f in ("k", "n_counters", "min_count", "bloom_bits_log2", "bloom_hashes",
              "bloom_block_log2", "seed"):
        assert getattr(best, f) == getattr(cfg, f)
    with kc.KmerCounter(best) as c:
        assert_matches_oracle(run_batch(c, dev), ref)
