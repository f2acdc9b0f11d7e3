"""The first shuffle level extracts each window's canonical key from two
packed words (w-1, w) and their reverse-complemented copies, left-aligned:
both orientations are taken with the window in the top 2k bits (the bases
after it below), and the key is the smaller 64-bit value shifted down by
64 - 2k.  This checks that rule, written with the same word operations, and
the right-aligned, masked form it replaced, against a base-by-base brute
force for every k and window end, random words and planted palindromes.  CPU
only.
"""
import random

M = (1 << 64) - 1


def rc_word(v):
    """The 32 bases of a packed word reversed and complemented (2-bit groups
    swapped within bytes, then bytes reversed)."""
    v = ~v & M
    v = ((v >> 2) & 0x3333333333333333) | ((v & 0x3333333333333333) << 2)
    v = ((v >> 4) & 0x0F0F0F0F0F0F0F0F) | ((v & 0x0F0F0F0F0F0F0F0F) << 4)
    return int.from_bytes(v.to_bytes(8, "little"), "big")


def left_aligned(pp, pc, qp, qc, k, j):
    sh = 66 + 2 * j - 2 * k
    f = ((pc << (sh - 64)) & M) if sh >= 64 else (((pp << sh) | (pc >> (64 - sh))) & M)
    sr = 62 - 2 * j
    r = ((qc << sr) & M) | (0 if sr == 0 else (qp >> (64 - sr)))
    return min(f, r) >> (64 - 2 * k)


def right_aligned(pp, pc, qp, qc, k, j):
    kmask = (1 << (2 * k)) - 1
    s = 62 - 2 * j
    f = ((((pc >> s) | (pp << (64 - s))) & M) if s else pc) & kmask
    s2 = 66 + 2 * j - 2 * k
    r = ((qc >> (s2 - 64)) if s2 >= 64 else (((qp >> s2) | (qc << (64 - s2))) & M)) & kmask
    return min(f, r)


def brute(bases, k, j):
    win = bases[33 + j - k:33 + j]
    f = r = 0
    for b in win:
        f = (f << 2) | b
    for b in reversed(win):
        r = (r << 2) | (3 - b)
    return min(f, r)


def _words(bases):
    pp = sum(b << (62 - 2 * i) for i, b in enumerate(bases[:32]))
    pc = sum(b << (62 - 2 * i) for i, b in enumerate(bases[32:]))
    return pp, pc


def test_rc_word_reverses_and_complements():
    rng = random.Random(3)
    bases = [rng.randrange(4) for _ in range(32)]
    w, _ = _words(bases + [0] * 32)
    want, _ = _words([3 - b for b in reversed(bases)] + [0] * 32)
    assert rc_word(w) == want


def test_both_forms_equal_brute_force():
    rng = random.Random(11)
    cases = 0
    for t in range(60):
        bases = [rng.randrange(4) for _ in range(64)]
        if t % 5 == 0:
            bases[32:] = bases[:32]  # repeated words
        pp, pc = _words(bases)
        qp, qc = rc_word(pp), rc_word(pc)
        for k in range(1, 32):
            for j in range(32):  # every window end in word w (k <= 31 fits the frame)
                want = brute(bases, k, j)
                assert left_aligned(pp, pc, qp, qc, k, j) == want, (k, j)
                assert right_aligned(pp, pc, qp, qc, k, j) == want, (k, j)
                cases += 1
    assert cases > 50000


def test_palindromic_windows():
    """Even k: a window equal to its own reverse complement (the two
    orientations tie in their top 2k bits)."""
    rng = random.Random(12)
    for k in range(2, 32, 2):
        for j in range(32):
            if 33 + j - k < 0:
                continue
            half = [rng.randrange(4) for _ in range(k // 2)]
            bases = [rng.randrange(4) for _ in range(64)]
            bases[33 + j - k:33 + j] = half + [3 - b for b in reversed(half)]
            pp, pc = _words(bases)
            qp, qc = rc_word(pp), rc_word(pc)
            assert left_aligned(pp, pc, qp, qc, k, j) == brute(bases, k, j)
