"""CPU check of the rule the read-start kernels use (k_rstart, k_rstart_batch,
read_start): the non-empty read that holds a word's first base (the word's
leader) writes the word's start bits with one store, scanning a bounded number
of later offset entries for the reads that begin in its last word; a start too
far from its leader, and a leader whose scan was cut short, or their bits in
atomically.  Every thread's writes are replayed on the CPU and checked against
the start set taken directly from the offsets (a base starts a read exactly
when it is the offset of a non-empty read), and a word stored to plainly must
have no other writer.
"""
import random

import pytest

SCAN = 64  # kStartScan


def thread_writes(offs, r, total, word0):
    """The stores ('put') and atomic ors ('or') that the thread of entry r
    makes, as (kind, word, bits)."""
    n = len(offs) - 1
    out = []
    o = offs[r]
    if r == n:
        return out
    e = offs[r + 1]
    if e == o:
        return out
    ws = o >> 5
    if (o & 31) and r >= SCAN and offs[r - SCAN] > (ws << 5):
        out.append(("or", word0 + ws, 1 << (o & 31)))
    wf, wl = (o + 31) >> 5, (e - 1) >> 5
    if wf > wl:
        return out
    if wf < wl and (o & 31) == 0:
        out.append(("put", word0 + wf, 1))
    lo = wl << 5
    bits = 1 if o == lo else 0
    cut = True
    for d in range(1, SCAN + 1):
        j = r + d
        if j >= n:
            cut = False
            break
        v = offs[j]
        if v < lo or v >= lo + 32:
            cut = False
            break
        if offs[j + 1] > v:
            bits |= 1 << (v - lo)
    if bits:
        out.append(("or" if cut else "put", word0 + wl, bits))
    return out


def replay(offs, total, word0, nwords):
    words = [0] * nwords
    writers = {}
    for r in range(len(offs)):
        for kind, w, bits in thread_writes(offs, r, total, word0):
            writers.setdefault(w, []).append(kind)
            words[w] = bits if kind == "put" else words[w] | bits
    for w, kinds in writers.items():
        if "put" in kinds:
            assert kinds == ["put"], (w, kinds)  # a plain store has no other writer
    return words


def direct(offs, word0, nwords):
    words = [0] * nwords
    for i in range(len(offs) - 1):
        if offs[i + 1] > offs[i]:
            p = offs[i]
            words[word0 + (p >> 5)] |= 1 << (p & 31)
    return words


def make_offsets(rng, n, lens):
    offs = [0]
    for _ in range(n):
        offs.append(offs[-1] + rng.choice(lens))
    return offs


@pytest.mark.parametrize("lens", [
    [100], [1, 2, 3, 5, 31, 32, 33], [0, 0, 0, 1, 7, 40], [0] * 40 + [1, 2],
    [64, 96, 128, 1000], [0, 31, 32, 33, 63, 64, 65], [0] * 200 + [3]])
def test_starts_match_the_offsets(lens):
    rng = random.Random(len(lens) * 7 + lens[-1])
    for trial in range(30):
        n = rng.randint(1, 400)
        offs = make_offsets(rng, n, lens)
        total = offs[-1]
        word0 = rng.choice([0, 3])
        nwords = word0 + (total + 31) // 32 + 1
        assert replay(offs, total, word0, nwords) == direct(offs, word0, nwords)


def test_long_runs_of_empty_reads_in_one_word():
    # hundreds of empty reads at offsets inside one word: starts past the
    # leader's scan are or-ed in, and the leader then ors too
    offs = [0, 5] + [9] * 300 + [10, 11] + [20] * 150 + [40, 100]
    total = offs[-1]
    nwords = (total + 31) // 32 + 1
    assert replay(offs, total, 0, nwords) == direct(offs, 0, nwords)
    kinds = [k for r in range(len(offs)) for k, w, _ in thread_writes(offs, r, total, 0) if w == 0]
    assert "or" in kinds and "put" not in kinds
