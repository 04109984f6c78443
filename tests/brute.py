"""Brute-force k-mer analysis for tiny inputs, written from the definition
with Python strings: every length-k substring is sliced out, its reverse
complement is built by reversing and complementing the string, and base-4
digits are read with int(s, 4).  It shares no code with the oracle (which
rolls 2-bit encodings in C++) and is used only to pin the oracle.

Definition followed: paper section "The Meraculous Assembly Pipeline" step 1
(chop reads into k-mers, count, drop rare ones, keep the neighbouring bases)
and section "Parallel k-mer analysis" (two arrays of four extension counters,
t_hq threshold); the readings (canonical form, quality gate, X/fork classes)
are the same as the oracle's and are listed in the design notes.
"""
from __future__ import annotations

DIGIT = {"A": "0", "C": "1", "G": "2", "T": "3"}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
BASES = "ACGT"
MASK64 = (1 << 64) - 1


def enc(w: str) -> int:
    return int("".join(DIGIT[c] for c in w.upper()), 4)


def revcomp(w: str) -> str:
    return "".join(COMP[c] for c in reversed(w.upper()))


def fmix64(x: int) -> int:
    """MurmurHash3 64-bit finalizer (Austin Appleby), in Python integers."""
    x &= MASK64
    x ^= x >> 33
    x = (x * 0xFF51AFD7ED558CCD) & MASK64
    x ^= x >> 33
    x = (x * 0xC4CEB9FE1A85EC53) & MASK64
    x ^= x >> 33
    return x


def owner(key: int, n_owners: int) -> int:
    """own(key) = floor(H * n / 2^64), H = (lo xor hi * m1) * m2 mod 2^64 (multiply-shift)."""
    hi, lo = key >> 64, key & MASK64
    h = ((lo ^ ((hi * 0x9E3779B97F4A7C15) & MASK64)) * 0xD1B54A32D192ED03) & MASK64
    return (h * n_owners) >> 64


def classify(t: list[int], ext_min: int) -> int:
    hits = [b for b in range(4) if t[b] >= ext_min]
    if not hits:
        return 5
    return hits[0] if len(hits) == 1 else 4


def brute(reads: list[tuple[str, list[int]]], k: int, qcut: int = 20, min_depth: int = 2, ext_min: int | None = None,
          forward_only: bool = False, keep_all: bool = False, n_owners: int = 1, own: int = 0,
          qual_offset: int = 0) -> dict[int, tuple]:
    """{key: (count, tl[4], tr[4], cls_l, cls_r)} for kept keys."""
    ext_min = min_depth if ext_min is None else ext_min
    table: dict[int, list] = {}
    for seq, qual in reads:
        L = len(seq)

        def hq(j):
            return 0 <= j < L and seq[j].upper() in DIGIT and qual[j] - qual_offset >= qcut

        for i in range(0, L - k + 1):
            w = seq[i:i + k]
            if any(c.upper() not in DIGIT for c in w):
                continue
            f, r = enc(w), enc(revcomp(w))
            if forward_only or f <= r:
                key = f
                left = seq[i - 1].upper() if hq(i - 1) else None
                right = seq[i + k].upper() if hq(i + k) else None
            else:
                key = r
                left = COMP[seq[i + k].upper()] if hq(i + k) else None
                right = COMP[seq[i - 1].upper()] if hq(i - 1) else None
            if n_owners > 1 and owner(key, n_owners) != own:
                continue
            rec = table.setdefault(key, [0, [0] * 4, [0] * 4])
            rec[0] += 1
            if left is not None:
                rec[1][BASES.index(left)] += 1
            if right is not None:
                rec[2][BASES.index(right)] += 1
    out = {}
    for key, (c, tl, tr) in table.items():
        if keep_all or c >= min_depth:
            out[key] = (c, tuple(tl), tuple(tr), classify(tl, ext_min), classify(tr, ext_min))
    return out


def decode(key: int, k: int) -> str:
    s = []
    for _ in range(k):
        s.append(BASES[key & 3])
        key >>= 2
    return "".join(reversed(s))


def card(reads: list[str], k: int, hll_p: int, sample_log2: int, heavy_log2: int, min_depth: int, heavy_min: int,
         forward_only: bool = False, n_owners: int = 1, own: int = 0) -> dict:
    """Cardinality pass from its definition, over Python strings: HyperLogLog registers (Flajolet et
    al. 2007: the top p bits of the key's 64-bit hash pick a register, which keeps the largest
    1 + leading-zero count of the remaining bits), the exact counts of the keys whose hash has
    `sample_log2` low zero bits, and per-key counts of the windows whose start index (in the
    concatenated reads) hashes to `heavy_log2` low zero bits."""
    regs = [0] * (1 << hll_p)
    sample: dict[int, int] = {}
    heavy: dict[int, int] = {}
    base, positions = 0, 0
    for seq in reads:
        for i in range(len(seq) - k + 1):
            w = seq[i:i + k]
            if any(c.upper() not in DIGIT for c in w):
                continue
            f, r = enc(w), enc(revcomp(w))
            key = f if forward_only or f <= r else r
            if n_owners > 1 and owner(key, n_owners) != own:
                continue
            positions += 1
            h = fmix64(fmix64((key >> 64) ^ 0xB7E151628AED2A6A) ^ (key & MASK64))
            j = h >> (64 - hll_p)
            rest = (h << hll_p) & MASK64
            rho = 64 - hll_p + 1 if rest == 0 else 64 - rest.bit_length() + 1
            regs[j] = max(regs[j], rho)
            if h % (1 << sample_log2) == 0:
                sample[key] = sample.get(key, 0) + 1
            if fmix64((base + i) ^ 0x452821E638D01377) % (1 << heavy_log2) == 0:
                heavy[key] = heavy.get(key, 0) + 1
        base += len(seq)
    return {"registers": regs, "sampled_distinct": len(sample),
            "sampled_kept": sum(1 for c in sample.values() if c >= min_depth),
            "heavy": sorted(x for x, c in heavy.items() if c >= heavy_min), "positions": positions}


def contigs(table: dict[int, tuple], k: int, forward_only: bool = False) -> list[str]:
    """Contigs of the UU k-mers of a brute-force table, with Python strings: two UU k-mers are
    linked when the extension of one spells the other and the other's extension spells the first
    back (a link from a side of a k-mer to the same side is not one); paths are spelled from an
    end and given as min(S, revcomp(S)), cycles from their smallest k-mer read forward."""
    uu = {key: (v[3], v[4]) for key, v in table.items() if v[3] < 4 and v[4] < 4}

    def spell(key):
        return "".join(BASES[(key >> (2 * (k - 1 - i))) & 3] for i in range(k))

    def canon(s):
        return s if forward_only else min(s, revcomp(s))

    def ext(s, side):
        c = canon(s)
        cl, cr = uu[enc(c)]
        if c == s:
            return BASES[cr] if side == "R" else BASES[cl]
        return COMP[BASES[cl]] if side == "R" else COMP[BASES[cr]]

    def step(s, d):
        t = s[1:] + ext(s, "R") if d == "R" else ext(s, "L") + s[:-1]
        if enc(canon(t)) not in uu:
            return None
        if (ext(t, "L") if d == "R" else ext(t, "R")) != (s[0] if d == "R" else s[-1]):
            return None
        if canon(t) == canon(s):
            leaves = "R" if (d == "R") == (s == canon(s)) else "L"
            arrives = "L" if (d == "R") == (t == canon(t)) else "R"
            if leaves == arrives:
                return None
        return t

    done, out = set(), []
    for key in sorted(uu):
        if key in done:
            continue
        start = spell(key)
        s, cycle = start, False
        while True:
            t = step(s, "L")
            if t is None:
                break
            if canon(t) == start:
                cycle = True
                break
            s = t
        if cycle:
            ring, s = [start], start
            while True:
                t = step(s, "R")
                if t is None or canon(t) == start:
                    break
                ring.append(canon(t))
                s = t
            m = min(ring)
            seq, s = m, m
            done.add(enc(m))
            while True:
                t = step(s, "R")
                if t is None or canon(t) == m:
                    break
                seq += t[-1]
                done.add(enc(canon(t)))
                s = t
            out.append(seq)
            continue
        seq = s
        done.add(enc(canon(s)))
        while True:
            t = step(s, "R")
            if t is None:
                break
            seq += t[-1]
            done.add(enc(canon(t)))
            s = t
        out.append(seq if forward_only else min(seq, revcomp(seq)))
    return sorted(out)
