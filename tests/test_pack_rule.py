"""CPU check of the four-bases-per-word rule the pack kernel uses (k_pack,
pack4): a byte's code is bits 1-2 of its ASCII value, the byte is a base
exactly when it equals "ACGT"[code], a nonzero byte of the difference is
detected without carries between bytes, and two multiplies gather the four
codes (first base on top) and the four invalid bits.  Checked against
byte-by-byte encoding (A0 C1 G2 T3; anything else invalid, coded 0) for every
byte value in every position and on random words.
"""
import random

M32 = 0xFFFFFFFF


def byte_perm(s0, s1, sel):
    """v_perm_b32 for selectors 0-7: byte i of the result is byte sel_i of
    the 64-bit value s0:s1 (s1 in the low half)."""
    both = (s0 << 32) | s1
    return sum(((both >> (8 * ((sel >> (8 * i)) & 0xFF))) & 0xFF) << (8 * i) for i in range(4))


def pack4(v):
    c = ((v >> 1) ^ (v >> 2)) & 0x03030303
    want = byte_perm(0, 0x54474341, c)
    z = v ^ want
    inv = (((((z & 0x7F7F7F7F) + 0x7F7F7F7F) & M32) | z) & 0x80808080) >> 7
    c &= ~(inv * 3) & M32
    return (((c * 0x40100401) & M32) >> 24) | (((((inv * 0x01020408) & M32) >> 24) & 0xF) << 8)


def bytewise(bs):
    code, inv = 0, 0
    for i, ch in enumerate(bs):
        ok = ch in b"ACGT"
        code = (code << 2) | (b"ACGT".index(ch) if ok else 0)
        inv |= (0 if ok else 1) << i
    return code | inv << 8


def test_every_byte_in_every_position():
    rng = random.Random(5)
    for pos in range(4):
        for b in range(256):
            for _ in range(3):
                bs = bytearray(rng.choice(b"ACGTN") for _ in range(4))
                bs[pos] = b
                assert pack4(int.from_bytes(bytes(bs), "little")) == bytewise(bytes(bs))


def test_random_words():
    rng = random.Random(6)
    for _ in range(50000):
        bs = bytes(rng.randrange(256) if rng.random() < 0.3 else rng.choice(b"ACGT")
                   for _ in range(4))
        assert pack4(int.from_bytes(bs, "little")) == bytewise(bs)
