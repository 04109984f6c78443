"""Helpers shared by the tests (not by the oracle or the GPU path)."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BASES = "ACGT"


def pack_reads(reads):
    """[(seq, qual list)] -> (ascii uint8, qual uint8, read_off int64)."""
    seqs = [s.encode() for s, _ in reads]
    quals = [bytes(q) for _, q in reads]
    off = np.zeros(len(reads) + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    ascii = np.frombuffer(b"".join(seqs), np.uint8).copy() if off[-1] else np.zeros(0, np.uint8)
    qual = np.frombuffer(b"".join(quals), np.uint8).copy() if off[-1] else np.zeros(0, np.uint8)
    return ascii, qual, off


def table_to_dict(t: dict) -> dict:
    """Table arrays -> {key_int: (count, tl, tr, cls_l, cls_r)}."""
    out = {}
    for i in range(len(t["count"])):
        key = (int(t["key_hi"][i]) << 64) | int(t["key_lo"][i])
        out[key] = (int(t["count"][i]), tuple(int(x) for x in t["tl"][i]), tuple(int(x) for x in t["tr"][i]),
                    int(t["cls_l"][i]), int(t["cls_r"][i]))
    return out


def enc(w: str) -> int:
    v = 0
    for c in w:
        v = v * 4 + BASES.index(c)
    return v


def read_golden(name: str) -> dict:
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            d.setdefault(key, []).append(vals)
    return d


def assert_tables_equal(a: dict, b: dict, what: str = ""):
    """Element-by-element equality of two sorted table dicts."""
    n_a, n_b = len(a["count"]), len(b["count"])
    assert n_a == n_b, "%s: %d vs %d records" % (what, n_a, n_b)
    for f in ("key_hi", "key_lo", "count", "tl", "tr", "cls_l", "cls_r"):
        x, y = np.asarray(a[f]), np.asarray(b[f])
        if not np.array_equal(x, y):
            bad = np.nonzero((x != y).reshape(len(x), -1).any(axis=1))[0]
            i = int(bad[0])
            raise AssertionError("%s: field %s differs at %d records; first at %d: %r vs %r (key %x:%x)" % (
                what, f, len(bad), i, x[i], y[i], int(a["key_hi"][i]), int(a["key_lo"][i])))


# ---- order-free table digest, written from its definition in include/hm_kmer.h
# (sum and xor over records of a chained MurmurHash3-finalizer hash)
def _fmix64(x):
    x = x ^ (x >> np.uint64(33))
    x = x * np.uint64(0xFF51AFD7ED558CCD)
    x = x ^ (x >> np.uint64(33))
    x = x * np.uint64(0xC4CEB9FE1A85EC53)
    x = x ^ (x >> np.uint64(33))
    return x


def table_digest(t: dict) -> tuple[int, int]:
    with np.errstate(over="ignore"):
        x = _fmix64(t["key_hi"].astype(np.uint64) ^ np.uint64(0x6A09E667F3BCC908))
        x = _fmix64(x ^ t["key_lo"].astype(np.uint64))
        x = _fmix64(x ^ t["count"].astype(np.uint64))
        for b in range(4):
            w = (t["tl"][:, b].astype(np.uint64) << np.uint64(32)) | t["tr"][:, b].astype(np.uint64)
            x = _fmix64(x ^ w)
        x = _fmix64(x ^ (t["cls_l"].astype(np.uint64) | (t["cls_r"].astype(np.uint64) << np.uint64(8))))
        s = int(np.sum(x, dtype=np.uint64)) if len(x) else 0
        xo = int(np.bitwise_xor.reduce(x)) if len(x) else 0
    return s, xo


def random_read_set(seed: int, n_reads: int, L_lo: int, L_hi: int, genome_len: int = 20000, err: float = 0.01,
                    n_rate: float = 0.0, lower_rate: float = 0.0):
    """Variable-length reads sampled from a random genome (both strands), with
    substitutions, optional N and lowercase bases, Phred 2..41."""
    rng = np.random.default_rng(seed)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), genome_len)
    comp = np.zeros(256, np.uint8)
    for a, b in zip(b"ACGT", b"TGCA"):
        comp[a] = b
    lens = rng.integers(L_lo, L_hi + 1, n_reads)
    seqs = []
    for L in lens:
        s = int(rng.integers(0, genome_len - L + 1))
        r = g[s:s + L].copy()
        if rng.random() < 0.5:
            r = comp[r[::-1]]
        e = rng.random(L) < err
        r[e] = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(e.sum()))
        if n_rate:
            r[rng.random(L) < n_rate] = ord("N")
        if lower_rate:
            lo = rng.random(L) < lower_rate
            r[lo] = r[lo] | 0x20
        seqs.append(r)
    off = np.zeros(n_reads + 1, np.int64)
    off[1:] = np.cumsum(lens)
    ascii = np.concatenate(seqs) if n_reads else np.zeros(0, np.uint8)
    qual = rng.integers(2, 42, int(off[-1])).astype(np.uint8)
    return ascii, qual, off
