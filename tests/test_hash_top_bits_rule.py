"""CPU check of the identity the shuffle kernels use to bucket keys
(mix64_top31): the top 31 bits of mix64(z) equal bits 31..1 of the high half
of mix64's second product, computed from three 32-bit multiplies, because
mix64's last step z ^ (z >> 31) leaves bits 63..33 unchanged.  Checked against
the oracle's mix64 on random and edge inputs.
"""
import random

import oracle

M64 = (1 << 64) - 1


def top31_rule(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    y = z ^ (z >> 27)
    ylo, yhi = y & 0xFFFFFFFF, y >> 32
    clo, chi = 0x133111EB, 0x94D049BB
    return (ylo * chi + yhi * clo + ((ylo * clo) >> 32)) & 0xFFFFFFFF


def test_top_bits_match_mix64():
    rng = random.Random(7)
    cases = [0, 1, M64, 1 << 63, (1 << 62) - 1] + [rng.getrandbits(64) for _ in range(20000)]
    for z in cases:
        assert top31_rule(z) >> 1 == oracle.mix64(z) >> 33, hex(z)
