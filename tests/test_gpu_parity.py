"""GPU path vs the CPU oracle, element by element, through the C ABI.

Every case prints its name, seed and shape before touching the GPU.
"""
import random

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import (assert_parity, assert_same_table, note, oracle_params, pack_reads,
                      random_reads, run_gpu, to_device, workload_chunks, workload_config)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def test_minimum_slice_keys_and_partitions():
    """Pass 1 alone: the stored key multiset equals the oracle's canonical
    windows, and every key sits in the partition given by the top bits of g."""
    note("case: minimum slice, plain_1mbp first 5000 reads")
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=5000)
    cfg = workload_config(w)
    db, do = to_device(b, o)
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        keys, part = c.debug_keys()
        st = c.stats()
    want = np.sort(oracle.enumerate_keys(oracle_params(cfg), b, o) >> np.uint64(1))
    got = keys & np.uint64((1 << 62) - 1)
    assert st["n_valid"] == want.size
    assert np.array_equal(np.sort(got), want)
    p_log2 = st["partitions_log2"]
    s0 = oracle.mix64(cfg.seed + 0x9E3779B97F4A7C15)
    sample = np.arange(0, got.size, 97)
    for i in sample:
        g = oracle.mix64(int(got[i]) ^ s0)
        assert int(part[i]) == g >> (64 - p_log2)
    assert part.max() < (1 << p_log2)


def test_plain_1mbp_full_parity():
    note("case: plain_1mbp full (20k reads x 100bp, k=31, m=2^24, h=3)")
    w, _, b, o = workload_chunks("plain_1mbp")
    cfg = workload_config(w)
    g, ref = assert_parity(cfg, [(b, o)])
    assert ref.stats["n_valid"] == 1_400_000
    note("stats: %s" % {k: g["stats"][k] for k in ("entries", "fp_singletons", "overflow_keys")})


PARAMS = [
    # k, m_log2, h, bl, p_log2, table_slots, nc, min_count, seed
    (31, 20, 4, 12, 0, 0, 1, 2, 1),
    (21, 22, 3, 19, 6, 0, 1, 2, 2),
    (15, 16, 2, 4, 0, 0, 1, 2, 3),      # Bloom blocks smaller than a word
    (9, 12, 8, 2, 0, 0, 1, 2, 4),       # h > block bits: repeated positions in S(x)
    (31, 24, 3, 19, 10, 0, 1, 3, 5),    # min_count 3, first-level fan-out 2^10
    (27, 26, 4, 16, 14, 0, 2, 2, 6),    # joint counters, two shuffle levels
    (1, 8, 2, 3, 0, 0, 1, 2, 7),
    (13, 10, 3, 5, 0, 64, 1, 2, 8),     # 64-slot tables: overflow path and its regrowth
    (31, 22, 4, 12, 12, 128, 1, 2, 9),  # 128-slot tables at 2^12 partitions
    (31, 24, 4, 10, 18, 64, 1, 2, 10),  # 2^18 partitions: runs of 0-1 keys per tile
    (31, 26, 4, 6, 20, 64, 1, 2, 12),   # 2^20 partitions: widest first level (2^10)
    (31, 27, 3, 6, 21, 64, 2, 2, 13),   # 2^21 partitions: widest second level (2^11)
    (31, 21, 4, 17, 0, 0, 1, 2, 14),    # 2^17-bit blocks: two per Bloom workgroup
    (25, 22, 3, 18, 5, 0, 1, 2, 15),    # blocks of two partitions, one per workgroup: flattened walk
    (9, 8, 3, 5, 0, 0, 1, 2, 16),       # one-word blocks, four per Bloom workgroup
]


@pytest.mark.parametrize("k,m,h,bl,pl,tl,nc,mc,seed", PARAMS)
def test_parameter_grid_parity(k, m, h, bl, pl, tl, nc, mc, seed):
    note("case: grid k=%d m=%d h=%d bl=%d p=%d t=%d nc=%d min=%d seed=%d"
         % (k, m, h, bl, pl, tl, nc, mc, seed))
    reads = random_reads(seed, 3000, 0, 160, genome_len=6000)
    cfg = kc.Config(k=k, bloom_bits_log2=m, bloom_hashes=h, bloom_block_log2=bl,
                    partitions_log2=pl, table_slots=tl, n_counters=nc, min_count=mc, seed=seed)
    b, o = pack_reads(reads)
    counters = None
    chunks = [(b, o)]
    if nc == 2:
        half = len(reads) // 2
        chunks = [pack_reads(reads[:half]), pack_reads(reads[half:])]
        counters = [0, 1]
    g, ref = assert_parity(cfg, chunks, counters)
    if tl == 64 and pl == 0:  # 64-slot tables at the minimum partition count overflow
        assert g["stats"]["overflow_keys"] > 0


@pytest.mark.parametrize("tile_log2", [10, 11, 12, 13])
def test_second_level_tile_sizes(tile_log2):
    """Second-level shuffle tiles of 2^10 to 2^13 keys (result-neutral): a
    first-level bucket is cut into more, shorter tiles, so every partition has
    more, shorter runs for the Bloom and count walks; the whole output equals
    the oracle's."""
    note("case: second-level tile 2^%d keys, 20000 reads of the 1 Mbp workload, 2^14 partitions"
         % tile_log2)
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=20000)
    cfg = workload_config(w, partitions_log2=14, shuffle_tile_log2=tile_log2)
    g, ref = assert_parity(cfg, [(b, o)])
    assert g["stats"]["partitions_log2"] == 14


def test_overflow_table_far_past_its_limit():
    """About 1.4·10^5 counted keys against 1024 table slots: the first overflow
    table (sized from n_valid / 256, a few thousand slots) takes a small
    fraction of them, so finalize grows it more than once; each void pass stops
    inserting once the table's limit is passed, and the last one equals the
    oracle."""
    note("case: overflow table far past its limit, 15000 reads x 100 bp from a 3e5 bp genome, "
         "16 partitions of 64 slots, seed 21")
    reads = random_reads(21, 15000, 100, 100, genome_len=300000)
    cfg = kc.Config(k=31, bloom_bits_log2=24, bloom_hashes=4, bloom_block_log2=16,
                    partitions_log2=4, table_slots=64, seed=21)
    g, ref = assert_parity(cfg, [pack_reads(reads)])
    st = g["stats"]
    note("overflow keys %d, retries %d" % (st["overflow_keys"], st["retries"]))
    assert st["overflow_keys"] > 100_000
    assert st["retries"] >= 2


def test_chunking_and_order_invariance():
    note("case: chunking invariance, 7 calls vs 1, plus shuffled read order")
    reads = random_reads(11, 4000, 20, 150, genome_len=5000)
    cfg = kc.Config(k=25, bloom_bits_log2=22, bloom_hashes=4, bloom_block_log2=16,
                    partitions_log2=9, seed=11)
    one = run_gpu(cfg, [pack_reads(reads)])
    cuts = [0, 1, 500, 501, 1700, 2900, 3999, 4000]
    many = run_gpu(cfg, [pack_reads(reads[a:b]) for a, b in zip(cuts[:-1], cuts[1:])])
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(reads))
    shuf = run_gpu(cfg, [pack_reads([reads[i] for i in perm])])
    for other in (many, shuf):
        assert_same_table(other["keys"], other["counts"], one["keys"], one["counts"])
        assert np.array_equal(other["b1"], one["b1"]) and np.array_equal(other["b2"], one["b2"])
        for key in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons"):
            assert other["stats"][key] == one["stats"][key]


def test_result_neutral_parameters():
    note("case: partitions / table size / fan-out change nothing")
    reads = random_reads(12, 3000, 30, 120, genome_len=4000)
    base = dict(k=19, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=14, seed=12)
    runs = [run_gpu(kc.Config(**base, partitions_log2=p, table_slots=t, scatter_bits=sb),
                    [pack_reads(reads)])
            for p, t, sb in [(0, 0, 0), (9, 0, 0), (12, 64, 0), (12, 0, 4), (6, 128, 3),
                             (9, 0, 5)]]  # last: two Bloom blocks per workgroup (bucket-limited)
    for r in runs[1:]:
        assert_same_table(r["keys"], r["counts"], runs[0]["keys"], runs[0]["counts"])
        assert np.array_equal(r["b1"], runs[0]["b1"]) and np.array_equal(r["b2"], runs[0]["b2"])
        assert r["stats"]["fp_singletons"] == runs[0]["stats"]["fp_singletons"]


def test_reverse_complement_invariance_on_gpu():
    note("case: reverse-complemented reads give the same table")
    reads = random_reads(13, 2000, 40, 100, genome_len=3000, nfrac=0.0)
    comp = str.maketrans("ACGT", "TGCA")
    cfg = kc.Config(k=31, bloom_bits_log2=20, bloom_hashes=4, bloom_block_log2=19, seed=13)
    a = run_gpu(cfg, [pack_reads(reads)])
    b = run_gpu(cfg, [pack_reads([r[::-1].translate(comp) for r in reads])])
    assert_same_table(a["keys"], a["counts"], b["keys"], b["counts"])
    assert np.array_equal(a["b2"], b["b2"])


def test_query_both_orientations_and_absent():
    import torch
    note("case: query, plain_1mbp 5000 reads")
    w, _, b, o = workload_chunks("plain_1mbp", n_reads=5000)
    cfg = workload_config(w)
    ref = oracle.count(oracle_params(cfg), b, o, want_bloom=False)
    table = dict(zip(ref.keys.tolist(), ref.counts[:, 0].tolist()))
    rng = np.random.default_rng(5)
    k = cfg.k
    present = ref.keys[rng.integers(0, ref.keys.size, 3000)]

    def rc(x):
        y = 0
        for j in range(k):
            y = (y << 2) | (3 - ((int(x) >> (2 * j)) & 3))
        return y
    flipped = np.array([rc(x) for x in present[:500]], np.uint64)
    rand = rng.integers(0, 1 << 62, 3000, dtype=np.uint64)
    q = np.concatenate([present, flipped, rand])
    db, do = to_device(b, o)
    with kc.KmerCounter(cfg) as c:
        c.insert_reads(db, do)
        c.finalize()
        out = c.query(torch.from_numpy(q.view(np.int64)).cuda()).cpu().numpy()
        for i, x in enumerate(q):
            xi = int(x)
            canon = min(xi, rc(xi))
            assert int(out[i, 0]) == table.get(canon, 0), (i, hex(xi))
        bad = torch.tensor([1 << 62], dtype=torch.int64, device="cuda")
        with pytest.raises(kc.KcError) as e:
            c.query(bad)
        assert e.value.status == kc.KC_ERR_INVALID_ARG


def test_joint_query_and_counters():
    import torch
    note("case: joint counters, query returns (normal, tumour)")
    normal = random_reads(21, 1500, 60, 100, genome_len=3000, nfrac=0.0)
    tumour = random_reads(22, 1500, 60, 100, genome_len=3000, nfrac=0.0)
    cfg = kc.Config(k=23, n_counters=2, bloom_bits_log2=20, bloom_hashes=4,
                    bloom_block_log2=15, seed=21)
    g, ref = assert_parity(cfg, [pack_reads(normal), pack_reads(tumour)], counters=[0, 1])
    with kc.KmerCounter(cfg) as c:
        for reads, t in ((normal, 0), (tumour, 1)):
            db, do = to_device(*pack_reads(reads))
            c.insert_reads(db, do, counter=t)
        c.finalize()
        out = c.query(torch.from_numpy(ref.keys[:2000].view(np.int64)).cuda()).cpu().numpy()
        assert np.array_equal(out.astype(np.uint32), ref.counts[:2000])


@pytest.mark.parametrize("tables,nc", [(100, 1), (1, 1), (3, 2), (255, 2)])
def test_forced_spill_keeps_results(tables, nc):
    """A table budget of `tables` partition tables: the other partitions are
    counted in waves and copied to pinned host memory, and every result (the
    exported table, queries on resident and spilled partitions, absent keys)
    matches the run without a budget."""
    import torch
    note("case: table budget of %d tables (of 256), %d counter(s): spill in waves" % (tables, nc))
    reads = random_reads(31, 3000, 50, 120, genome_len=6000)
    cfg = kc.Config(k=27, n_counters=nc, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=14,
                    partitions_log2=8, table_slots=256, seed=31)
    chunks = [pack_reads(reads[:1500]), pack_reads(reads[1500:])]
    counters = [0, 1] if nc == 2 else [0, 0]
    per_table = 256 * (8 + 4 * nc)
    cfg.hbm_table_budget_bytes = per_table * tables
    # table, Bloom levels and statistics of the budgeted run against the oracle
    _, ref = assert_parity(cfg, chunks, counters=counters)
    full = {"keys": ref.keys, "counts": ref.counts.reshape(-1, nc)}
    rng = np.random.default_rng(tables)
    absent = rng.integers(0, 1 << (2 * cfg.k), 4000, dtype=np.uint64)
    absent = absent[~np.isin(absent, full["keys"])]
    qk = np.concatenate([full["keys"], absent])
    want = np.zeros((qk.size, nc), np.uint32)
    want[:full["keys"].size] = full["counts"]
    with kc.KmerCounter(cfg) as c:
        for (b, o), t in zip(chunks, counters):
            db, do = to_device(b, o)
            c.insert_reads(db, do, counter=t)
        st = c.finalize()
        assert st["spilled_partitions"] == 256 - tables
        assert st["spilled_bytes"] == (256 - tables) * per_table
        keys, counts = c.export()
        assert_same_table(keys, counts, full["keys"], full["counts"])
        q = torch.from_numpy(qk.view(np.int64)).cuda()
        out = c.query(q).cpu().numpy().astype(np.uint32).reshape(-1, nc)
        assert np.array_equal(out, want)
        # explicit spill of a resident partition (the highest ones stay in HBM)
        moved = c.spill(255)
        assert moved == per_table
        assert c.spill(255) == 0 and c.spill(0) == 0
        out = c.query(q).cpu().numpy().astype(np.uint32).reshape(-1, nc)
        assert np.array_equal(out, want)
        keys, counts = c.export()
        assert_same_table(keys, counts, full["keys"], full["counts"])
        assert c.stats()["spilled_partitions"] == 257 - tables


def test_edge_inputs():
    note("case: empty reads, reads shorter than k, all-invalid reads, empty insert")
    cfg = kc.Config(k=11, bloom_bits_log2=16, bloom_hashes=3, bloom_block_log2=12, seed=41)
    reads = ["", "ACG", "", "NNNNNNNNNNNNNNNNNNNN", "ACGTACGTACGTACGT", "", "ACGTACGTACGTACGTT",
             "acgtacgtacgtacgt", "A" * 50, "T" * 40, ""]
    assert_parity(cfg, [pack_reads(reads), pack_reads([]), pack_reads([""])])
    assert_parity(cfg, [])


def test_bad_offsets_and_state_errors():
    import torch
    note("case: invalid offsets and out-of-order calls are rejected")
    cfg = kc.Config(k=11, bloom_bits_log2=16, bloom_hashes=3, bloom_block_log2=12, seed=42)
    b, o = pack_reads(["ACGTACGTACGTAC", "GGGGCCCCAAAATTTT"])
    with kc.KmerCounter(cfg) as c:
        db = torch.from_numpy(b).cuda()
        for bad in (np.array([0, 20, 10], np.int64), np.array([1, 5, 30], np.int64),
                    np.array([0, 5, 29], np.int64)):
            with pytest.raises(kc.KcError) as e:
                c.insert_reads(db, torch.from_numpy(bad).cuda())
            assert e.value.status == kc.KC_ERR_INVALID_ARG
        c.insert_reads(db, torch.from_numpy(o.view(np.int64)).cuda())
        with pytest.raises(kc.KcError) as e:
            c.export()
        assert e.value.status == kc.KC_ERR_BAD_STATE
        c.finalize()
        with pytest.raises(kc.KcError) as e:
            c.insert_reads(db, torch.from_numpy(o.view(np.int64)).cuda())
        assert e.value.status == kc.KC_ERR_BAD_STATE
        c.reset()
        c.insert_reads(db, torch.from_numpy(o.view(np.int64)).cuda())
        st = c.finalize()
        assert st["n_valid"] == (14 - 11 + 1) + (16 - 11 + 1)


@pytest.mark.gpu
@pytest.mark.parametrize("nc,pl", [(1, 4), (2, 6)])
def test_contended_tables_parity(nc, pl):
    """Few distinct k-mers seen from every wave at once: reads from a 300-base
    genome at ~6,000x coverage, homopolymer and dinucleotide and trinucleotide
    repeats, so the same table buckets are read while other waves insert into
    them (the count pass reads buckets without atomics): 280 distinct keys
    over 1.2 million occurrences, the largest count about 40,000; one and two
    counters, 16 and 64 partitions."""
    note("case: contended tables nc=%d partitions=2^%d" % (nc, pl))
    rng = random.Random(77 + nc)
    genome = "".join(rng.choice("ACGT") for _ in range(300))
    comp = str.maketrans("ACGT", "TGCA")
    reads = []
    for i in range(18000):
        L = rng.randint(60, 120)
        st = rng.randint(0, len(genome) - L)
        r = genome[st:st + L]
        reads.append(r[::-1].translate(comp) if i & 1 else r)
    for unit in ("A", "T", "C", "AC", "GT", "AGC", "TTG"):
        for _ in range(300):
            L = rng.randint(40, 150)
            reads.append((unit * (L // len(unit) + 1))[:L])
    rng.shuffle(reads)
    half = len(reads) // 2
    cfg = kc.Config(k=31, n_counters=nc, bloom_bits_log2=20, bloom_hashes=4, bloom_block_log2=14,
                    seed=91 + nc, partitions_log2=pl)
    if nc == 1:
        assert_parity(cfg, [pack_reads(reads)])
    else:
        assert_parity(cfg, [pack_reads(reads[:half]), pack_reads(reads[half:])], counters=[0, 1])
