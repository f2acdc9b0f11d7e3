"""The served workload's per-request counting parameters and the choice of
requests checked against the oracle (host logic, no GPU).

A request of n reads of length L has n * max(0, L - k + 1) k-mer windows; its
Bloom filter has 2^m bits with m = clamp(ceil(log2(8 * windows)), 20, 34),
and its partition count (result-neutral) is about one per 2^13 bases, at
least one per Bloom block.
"""
import math

import numpy as np

import synth
from digest import served_subset


def test_request_bloom_size_rule():
    w = synth.WORKLOADS["served_300mbp"]
    assert (w.lmax, w.k, w.bloom_block_log2) == (100, 31, 16)
    # hand-worked: 10^4 reads -> 7·10^5 windows, 8x = 5.6·10^6 -> 2^23 (8388608)
    assert w.request_params(10_000)[:2] == (700_000, 23)
    # 5·10^6 reads -> 3.5·10^8 windows, 8x = 2.8·10^9 -> 2^32 (4294967296)
    assert w.request_params(5_000_000)[:2] == (350_000_000, 32)
    # tiny requests clamp at 2^20 bits
    assert w.request_params(2)[1] == 20
    # across a power of two: 8 * 70 * 119837 = 67108720 <= 2^26, 8 * 70 * 119838 = 67109280 > 2^26
    assert w.request_params(119_837)[1] == 26
    assert w.request_params(119_838)[1] == 27


def test_request_partitions_rule():
    w = synth.WORKLOADS["served_300mbp"]
    for n in (10, 10_000, 123_457, 2_000_000, 5_000_000):
        _, m, pl = w.request_params(n)
        assert pl >= m - w.bloom_block_log2  # at least one partition per Bloom block
        assert pl >= round(math.log2(max(1, n * w.lmax) / 8192))


def test_served_subset_takes_the_largest_and_distinct_others():
    w = synth.WORKLOADS["served_300mbp"]
    sizes = w.request_plan()[w.warmup_requests:, 0]
    pick = served_subset(sizes, seed=w.seed)
    assert len(pick) == 16 == len(set(pick))
    assert pick == sorted(pick)
    assert int(np.argmax(sizes)) in pick
    assert all(0 <= i < sizes.size for i in pick)
    assert served_subset(sizes, seed=w.seed) == pick  # seeded
