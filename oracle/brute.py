"""Pure-Python brute force of the counting definitions, for tiny inputs only.

TEST INFRASTRUCTURE ONLY.  A second, independent reading of the definitions the
C oracle implements, written on strings rather than integers:

* k-mers of a read are its length-k substrings (paper Sec. II-A); windows with
  a byte outside ``ACGT`` are skipped; no window spans two reads;
* the canonical k-mer is the lexicographically smaller of the window and its
  reverse complement (with A<C<G<T this equals the smaller 2-bit code, code
  A=0 C=1 G=2 T=3, first base most significant);
* count(x) = number of occurrences; the table keeps count >= min_count
  (Sec. II-B, Count unit);
* stems (Sec. II-A): a k-mer without its first and last base; stem items
  (Sec. III-D): per canonical stem (lexicographically smaller of the stem and
  its reverse complement), the counts of the k-mers read as a + stem + b in
  that orientation, at slot 4*rank(a) + rank(b), saturated to 65535;
* Filter-unit lookup (Sec. II-B): per read, the windows whose canonical
  k-mer has tumour count >= tumour_min and normal count <= normal_max in the
  final table (absent: 0 and 0; one counter: normal 0, tumour = the count);
* Bloom levels (Sec. III, Prune unit) from explicit per-bit hit counters:
  hits(b) = sum over occurrences of x of [b in S(x)], B1 = hits >= 1,
  B2 = hits >= 2; a key passes iff every bit of S(x) is in B2; F = keys seen
  once that pass (Sec. III, Unify unit removes them).
"""
from __future__ import annotations

from collections import Counter, defaultdict

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_COMP = str.maketrans("ACGT", "TGCA")


def mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def encode(s: str) -> int:
    """2-bit code of a k-mer string, first base most significant."""
    v = 0
    for ch in s:
        v = v * 4 + "ACGT".index(ch)
    return v


def decode(x: int, k: int) -> str:
    return "".join("ACGT"[(x >> (2 * (k - 1 - j))) & 3] for j in range(k))


def revcomp(s: str) -> str:
    return s[::-1].translate(_COMP)


def canonical(s: str) -> str:
    return min(s, revcomp(s))


def windows(read: str, k: int):
    for i in range(len(read) - k + 1):
        w = read[i:i + k]
        if all(c in "ACGT" for c in w):
            yield w


def salts(seed: int, h: int):
    return [mix64((seed + (i + 1) * GAMMA) & M64) for i in range(h + 1)]


def bloom_set(x: int, m_log2: int, h: int, block_log2: int, seed: int) -> set:
    """S(x): h positions a + i*b (mod the block size) in x's block, where a
    and b are the first two block_log2-bit fields of mix64(x ^ s_1), read off
    its binary digits (double hashing)."""
    s = salts(seed, h)
    sb = m_log2 - block_log2
    g = mix64(x ^ s[0])
    block = (g >> (64 - sb)) if sb > 0 else 0
    digits = format(mix64(x ^ s[1]), "064b")
    a = int(digits[:block_log2], 2)
    b = int(digits[block_log2:2 * block_log2], 2)
    size = 1 << block_log2
    return {block * size + (a + i * b) % size for i in range(h)}


def count(reads, k, m_log2, h, block_log2, seed, min_count=2, tags=None, n_counters=1):
    """Brute-force count.  ``reads`` is a list of str; ``tags`` the counter of each read."""
    per = defaultdict(lambda: [0] * n_counters)
    n_valid = 0
    for r, read in enumerate(reads):
        t = tags[r] if tags is not None else 0
        for w in windows(read, k):
            per[encode(canonical(w))][t] += 1
            n_valid += 1
    hits = Counter()
    sets = {}
    for x, cs in per.items():
        sets[x] = bloom_set(x, m_log2, h, block_log2, seed)
        for b in sets[x]:
            hits[b] += sum(cs)
    b1 = {b for b, v in hits.items() if v >= 1}
    b2 = {b for b, v in hits.items() if v >= 2}
    table, n_pass, fp = {}, 0, 0
    for x, cs in per.items():
        c = sum(cs)
        passed = sets[x] <= b2
        if passed:
            n_pass += c
            fp += c == 1
        if c >= min_count:
            table[x] = tuple(cs)
    stats = dict(n_valid=n_valid, n_distinct=len(per), n_pass=n_pass, entries=len(table),
                 sum_counts=sum(sum(v) for v in table.values()), fp_singletons=fp,
                 b1_pop=len(b1), b2_pop=len(b2))
    return table, b1, b2, stats


def stem_items(table: dict, k: int, n_counters: int = 1) -> dict:
    """table: canonical k-mer string -> counts tuple (the final table).
    Returns canonical stem string -> [[16 counts] per counter]."""
    rank = {c: i for i, c in enumerate("ACGT")}
    out = {}
    for kmer, cs in table.items():
        assert len(kmer) == k
        stem = kmer[1:-1]
        rstem = revcomp(stem)
        if stem <= rstem:
            canon, a, b = stem, kmer[0], kmer[-1]
        else:
            r = revcomp(kmer)
            canon, a, b = rstem, r[0], r[-1]
        item = out.setdefault(canon, [[0] * 16 for _ in range(n_counters)])
        for t in range(n_counters):
            item[t][4 * rank[a] + rank[b]] = min(cs[t], 65535)
    return out


def filter_reads(table: dict, reads, k: int, tumour_min: int, normal_max: int,
                 n_counters: int = 2) -> list:
    """table: canonical k-mer code -> counts tuple (the final table)."""
    out = []
    for read in reads:
        sel = 0
        for w in windows(read, k):
            cs = table.get(encode(canonical(w)), (0,) * n_counters)
            normal, tumour = (cs[0], cs[1]) if n_counters == 2 else (0, cs[0])
            sel += tumour >= tumour_min and normal <= normal_max
        out.append(sel)
    return out
