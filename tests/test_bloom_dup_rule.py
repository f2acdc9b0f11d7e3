"""The Bloom pass marks repeated positions of S(x) with a closed form instead
of comparing positions pairwise: with positions a + i*b mod 2^bl (double
hashing, i < h <= 8), position i equals an earlier one exactly when b has at
least bl - floor(log2 i) trailing zero bits (b = 0 counting as 32).  This
checks the rule against the pairwise comparison for every b at small block
sizes and for sampled b up to the largest block size.  CPU only.
"""
import numpy as np


def _tz(b):
    return 32 if b == 0 else (b & -b).bit_length() - 1


def _rule(b, i, bl):
    lg = 2 if i >= 4 else 1 if i >= 2 else 0
    return i > 0 and _tz(b) + lg >= bl


def _pairwise(a, b, i, bl):
    m = (1 << bl) - 1
    return any(((a + i * b) & m) == ((a + j * b) & m) for j in range(i))


def test_rule_equals_pairwise_for_every_b_at_small_blocks():
    for bl in range(1, 11):
        for b in range(1 << bl):
            for i in range(8):
                assert _rule(b, i, bl) == _pairwise(5, b, i, bl), (bl, b, i)


def test_rule_equals_pairwise_for_sampled_b_up_to_the_largest_block():
    rng = np.random.default_rng(9)
    for bl in range(11, 20):
        bs = [0, 1 << (bl - 1), 1 << (bl - 2), 3 << (bl - 2), 1 << (bl - 3)]
        bs += [int(v) for v in rng.integers(0, 1 << bl, 200)]
        for b in bs:
            a = int(rng.integers(0, 1 << bl))
            for i in range(8):
                assert _rule(b, i, bl) == _pairwise(a, b, i, bl), (bl, b, i)
