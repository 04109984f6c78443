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
