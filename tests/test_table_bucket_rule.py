"""Partition tables are cut into aligned buckets of four slots, and the count
pass reads a key's home bucket with two 16-byte LDS loads that are not atomic
against another wave's 64-bit CAS on one of its slots.  Such a read can see a
slot torn: one 32-bit half already holding the new key, the other still all
ones (the empty slot is 2^64 - 1).  The kernel takes a slot whose value has a
32-bit half of all ones as open (empty or being written), never as holding x
or another key.  That is sound because no canonical key has a 32-bit half of
all ones: the high half is below 2^30 (x < 2^62), and a key whose last 16
bases are all T has a reverse complement that starts with 16 A bases, which is
smaller whenever k <= 31.  This checks that claim base by base (every window
ending in 16 T bases for k up to 22, random ones above, random windows for every
k) and the bucket alignment of home slots.  CPU only.
"""
import itertools
import random

CODE = {"A": 0, "C": 1, "G": 2, "T": 3}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
ONES = 0xFFFFFFFF


def enc(s):
    v = 0
    for b in s:
        v = (v << 2) | CODE[b]
    return v


def canonical(s):
    rc = "".join(COMP[b] for b in reversed(s))
    return min(enc(s), enc(rc))


def halves_open(v):
    """The kernel's test for a slot that is empty or torn."""
    return max(v & ONES, v >> 32) == ONES


def test_no_canonical_key_ending_in_sixteen_t_has_an_all_ones_half():
    rng = random.Random(5)
    checked = 0
    for k in range(16, 32):
        n = k - 16
        if 4 ** n <= 4096:
            prefixes = ("".join(p) for p in itertools.product("ACGT", repeat=n))
        else:
            prefixes = ("".join(rng.choice("ACGT") for _ in range(n)) for _ in range(2000))
        for p in prefixes:
            x = canonical(p + "T" * 16)
            assert x < 1 << 62
            assert not halves_open(x), (k, p)
            checked += 1
    assert checked > 20000


def test_random_canonical_keys_have_no_all_ones_half():
    rng = random.Random(6)
    for k in range(1, 32):
        for _ in range(400):
            s = "".join(rng.choice("ACGT") for _ in range(k))
            x = canonical(s)
            assert not halves_open(x), (k, s)
        # runs of T and A at either end, the only way to approach all ones
        for a in range(0, k + 1):
            s = "A" * a + "T" * (k - a)
            assert not halves_open(canonical(s)), (k, s)
            s = "T" * a + "A" * (k - a)
            assert not halves_open(canonical(s)), (k, s)


def test_torn_slots_read_as_open_and_never_as_a_key():
    rng = random.Random(7)
    empty = (1 << 64) - 1
    assert halves_open(empty)
    for _ in range(2000):
        k = rng.randrange(1, 32)
        y = canonical("".join(rng.choice("ACGT") for _ in range(k)))
        for torn in ((y & ~ONES) | ONES, (ONES << 32) | (y & ONES)):
            assert halves_open(torn)
            assert torn != y


def home_slot(th, cap):
    """First slot of the key's bucket: the top 32 bits of th scaled to the
    cap / 4 buckets."""
    return (((th >> 32) * (cap // 4)) >> 32) * 4


def test_home_slots_are_bucket_aligned_and_cover_the_buckets():
    rng = random.Random(8)
    for cap in (64, 128, 3456, 3840, 8192):
        seen = set()
        for _ in range(20000):
            h = home_slot(rng.getrandbits(64), cap)
            assert h % 4 == 0 and h + 3 < cap
            seen.add(h)
        if cap <= 3840:
            assert len(seen) == cap // 4  # every bucket is somebody's home
        assert home_slot(0, cap) == 0 and home_slot((1 << 64) - 1, cap) == cap - 4
