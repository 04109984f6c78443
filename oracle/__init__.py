"""TEST INFRASTRUCTURE -- Python loader for the CPU oracle (kmer_oracle.cpp).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU path never imports it and shares no code with
it.  ``run()`` returns the sorted, depth-filtered table of k-mer analysis as
defined in the paper's sections "The Meraculous Assembly Pipeline" (step 1)
and "Parallel k-mer analysis"; see kmer_oracle.cpp for the readings taken
where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmer_oracle.cpp")
_SO = os.path.join(_HERE, "libkmer_oracle.so")

FORWARD_ONLY = 1
KEEP_ALL = 2
SPLIT_READS = 4
SORT_COUNT = 8

CLS_FORK = 4
CLS_X = 5


class OrcParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("qual_offset", ctypes.c_int32), ("qcut", ctypes.c_int32),
                ("min_depth", ctypes.c_uint32), ("ext_min", ctypes.c_uint32), ("n_owners", ctypes.c_uint32),
                ("owner", ctypes.c_uint32), ("n_shards", ctypes.c_uint32), ("shard", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("n_threads", ctypes.c_int32)]


class OrcCardParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("flags", ctypes.c_uint32), ("n_owners", ctypes.c_uint32),
                ("owner", ctypes.c_uint32), ("hll_p", ctypes.c_int32), ("sample_log2", ctypes.c_uint32),
                ("heavy_log2", ctypes.c_uint32), ("min_depth", ctypes.c_uint32), ("heavy_min", ctypes.c_uint32),
                ("n_threads", ctypes.c_int32)]


class OrcCardResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("sampled_distinct", ctypes.c_uint64),
                ("sampled_kept", ctypes.c_uint64), ("n_heavy", ctypes.c_uint64), ("positions", ctypes.c_int64)]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (host code only)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        build()
        L = ctypes.CDLL(_SO)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_run.argtypes = [u8p, u8p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, ctypes.POINTER(OrcParams),
                              ctypes.POINTER(ctypes.c_void_p)]
        L.orc_run.restype = ctypes.c_int64
        L.orc_fetch.argtypes = [ctypes.c_void_p, ctypes.c_uint32] + [ctypes.c_void_p] * 7
        L.orc_fetch.restype = None
        L.orc_acc_new.argtypes = [ctypes.POINTER(OrcParams)]
        L.orc_acc_new.restype = ctypes.c_void_p
        L.orc_acc_add.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
        L.orc_acc_add.restype = ctypes.c_int
        L.orc_acc_finish.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_acc_finish.restype = ctypes.c_int64
        L.orc_acc_free.argtypes = [ctypes.c_void_p]
        L.orc_acc_free.restype = None
        L.orc_positions.argtypes = [ctypes.c_void_p]
        L.orc_positions.restype = ctypes.c_int64
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_free.restype = None
        L.orc_owner.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_owner.restype = ctypes.c_uint32
        L.orc_shard.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_shard.restype = ctypes.c_uint32
        L.orc_part_many.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_int32, ctypes.c_void_p]
        L.orc_part_many.restype = None
        L.orc_card.argtypes = [u8p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, ctypes.POINTER(OrcCardParams),
                               ctypes.c_void_p, ctypes.POINTER(OrcCardResult), ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_uint64]
        L.orc_card.restype = ctypes.c_int
        L.orc_contigs.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                          ctypes.POINTER(ctypes.c_int64)]
        L.orc_contigs.restype = ctypes.c_void_p
        L.orc_contigs_bases.argtypes = [ctypes.c_void_p]
        L.orc_contigs_bases.restype = ctypes.c_int64
        L.orc_contigs_fetch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_contigs_fetch.restype = None
        L.orc_contigs_free.argtypes = [ctypes.c_void_p]
        L.orc_contigs_free.restype = None
        _LIB = L
    return _LIB


def _params(k, qcut, min_depth, ext_min, n_owners, owner, n_shards, shard, qual_offset, forward_only, keep_all,
            n_threads, split_reads, sort_count=False):
    ext_min = min_depth if ext_min is None else ext_min
    p = OrcParams(k, qual_offset, qcut, min_depth, ext_min, n_owners, owner, n_shards, shard,
                  (FORWARD_ONLY if forward_only else 0) | (KEEP_ALL if keep_all else 0) |
                  (SPLIT_READS if split_reads else 0) | (SORT_COUNT if sort_count else 0), n_threads)
    return p, ext_min


def _fetch(h, n, ext_min) -> dict:
    L = lib()
    out = {"key_hi": np.empty(n, np.uint64), "key_lo": np.empty(n, np.uint64), "count": np.empty(n, np.uint32),
           "tl": np.empty((n, 4), np.uint32), "tr": np.empty((n, 4), np.uint32), "cls_l": np.empty(n, np.uint8),
           "cls_r": np.empty(n, np.uint8)}
    try:
        L.orc_fetch(h, ext_min, *(out[x].ctypes.data for x in ("key_hi", "key_lo", "count", "tl", "tr", "cls_l",
                                                             "cls_r")))
        out["positions"] = int(L.orc_positions(h))
    finally:
        L.orc_free(h)
    return out


class Accumulator:
    """The oracle over reads given in batches (e.g. a read set too large to hold on the host at
    once): add() counts a batch into the same state, finish() filters and sorts.  By additivity
    of unfiltered tables the result equals run() over the concatenated batches.  Same keyword
    arguments as run(); 'seconds' adds up the time spent in add() and finish()."""

    def __init__(self, k: int, qcut: int = 20, min_depth: int = 2, ext_min: int | None = None, n_owners: int = 1,
                 owner: int = 0, n_shards: int = 1, shard: int = 0, qual_offset: int = 0, forward_only: bool = False,
                 keep_all: bool = False, n_threads: int = 1, split_reads: bool = False, sort_count: bool = False):
        p, self.ext_min = _params(k, qcut, min_depth, ext_min, n_owners, owner, n_shards, shard, qual_offset,
                                  forward_only, keep_all, n_threads, split_reads, sort_count)
        self._h = lib().orc_acc_new(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle: bad parameters")
        self.seconds = 0.0

    def add(self, ascii: np.ndarray, qual: np.ndarray, read_off: np.ndarray):
        ascii = np.ascontiguousarray(ascii, dtype=np.uint8)
        qual = np.ascontiguousarray(qual, dtype=np.uint8)
        read_off = np.ascontiguousarray(read_off, dtype=np.int64)
        if read_off[-1] > ascii.size or read_off[-1] > qual.size:
            raise ValueError("read offsets exceed the base arrays")
        t0 = time.perf_counter()
        rc = lib().orc_acc_add(self._h, ascii.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               qual.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               read_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), read_off.size - 1)
        self.seconds += time.perf_counter() - t0
        if rc != 0:
            raise ValueError("oracle failed with code %d" % rc)

    def finish(self) -> dict:
        h = ctypes.c_void_p()
        t0 = time.perf_counter()
        n = lib().orc_acc_finish(self._h, ctypes.byref(h))
        self._h = None
        self.seconds += time.perf_counter() - t0
        if n < 0:
            raise ValueError("oracle failed with code %d" % n)
        out = _fetch(h, n, self.ext_min)
        out["seconds"] = self.seconds
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_acc_free(self._h)
            self._h = None


def run(ascii: np.ndarray, qual: np.ndarray, read_off: np.ndarray, k: int, qcut: int = 20, min_depth: int = 2,
        ext_min: int | None = None, n_owners: int = 1, owner: int = 0, n_shards: int = 1, shard: int = 0,
        qual_offset: int = 0, forward_only: bool = False, keep_all: bool = False, n_threads: int = 1,
        split_reads: bool = False, sort_count: bool = False) -> dict:
    """Oracle table as a dict of numpy arrays sorted by (key_hi, key_lo):
    key_hi, key_lo (uint64), count (uint32), tl, tr (uint32, n x 4),
    cls_l, cls_r (uint8: 0..3 unique base, 4 fork, 5 none), plus
    'positions' (valid windows scanned) and 'seconds' (wall time of the run)."""
    ascii = np.ascontiguousarray(ascii, dtype=np.uint8)
    qual = np.ascontiguousarray(qual, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    n_reads = read_off.size - 1
    if read_off[-1] > ascii.size or read_off[-1] > qual.size:
        raise ValueError("read offsets exceed the base arrays")
    p, ext_min = _params(k, qcut, min_depth, ext_min, n_owners, owner, n_shards, shard, qual_offset, forward_only,
                         keep_all, n_threads, split_reads, sort_count)
    h = ctypes.c_void_p()
    L = lib()
    t0 = time.perf_counter()
    n = L.orc_run(ascii.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                  qual.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                  read_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_reads, ctypes.byref(p), ctypes.byref(h))
    secs = time.perf_counter() - t0
    if n < 0:
        raise ValueError("oracle failed with code %d" % n)
    out = _fetch(h, n, ext_min)
    out["seconds"] = secs
    return out


def _parts(key_hi, key_lo, n, which):
    hi = np.ascontiguousarray(key_hi, dtype=np.uint64)
    lo = np.ascontiguousarray(key_lo, dtype=np.uint64)
    out = np.empty(hi.size, np.uint32)
    lib().orc_part_many(hi.ctypes.data, lo.ctypes.data, hi.size, n, which, out.ctypes.data)
    return out


def owner_of(key_hi: np.ndarray, key_lo: np.ndarray, n_owners: int) -> np.ndarray:
    """own(key) for every record (method-defined owner map)."""
    return _parts(key_hi, key_lo, n_owners, 0)


def shard_of(key_hi: np.ndarray, key_lo: np.ndarray, n_shards: int) -> np.ndarray:
    """Test-sampling shard of every record (independent of the owner map)."""
    return _parts(key_hi, key_lo, n_shards, 1)


def uu_mask(t: dict) -> np.ndarray:
    """UU records: unique high-quality extension on both sides."""
    return (t["cls_l"] < 4) & (t["cls_r"] < 4)


def card(ascii: np.ndarray, read_off: np.ndarray, k: int, hll_p: int = 14, sample_log2: int = 10,
         heavy_log2: int = 8, min_depth: int = 2, heavy_min: int = 64, n_owners: int = 1, owner: int = 0,
         forward_only: bool = False, n_threads: int = 1, heavy_cap: int = 1 << 16) -> dict:
    """Cardinality pass over the reads (see orc_card in kmer_oracle.cpp): HyperLogLog registers and
    estimate of the distinct owned k-mers, the exact distinct sample's size and kept count, and the
    sorted heavy-hitter keys (at most heavy_cap returned; 'n_heavy' is the full number)."""
    ascii = np.ascontiguousarray(ascii, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    if read_off[-1] > ascii.size:
        raise ValueError("read offsets exceed the base array")
    p = OrcCardParams(k, FORWARD_ONLY if forward_only else 0, n_owners, owner, hll_p, sample_log2, heavy_log2,
                      min_depth, heavy_min, n_threads)
    regs = np.zeros(1 << hll_p, np.uint32)
    hh = np.zeros(heavy_cap, np.uint64)
    hl = np.zeros(heavy_cap, np.uint64)
    res = OrcCardResult()
    t0 = time.perf_counter()
    rc = lib().orc_card(ascii.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                        read_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), read_off.size - 1, ctypes.byref(p),
                        regs.ctypes.data, ctypes.byref(res), hh.ctypes.data, hl.ctypes.data, heavy_cap)
    secs = time.perf_counter() - t0
    if rc != 0:
        raise ValueError("oracle cardinality pass failed with code %d" % rc)
    n = min(int(res.n_heavy), heavy_cap)
    return {"registers": regs, "estimate": res.estimate, "sampled_distinct": int(res.sampled_distinct),
            "sampled_kept": int(res.sampled_kept), "n_heavy": int(res.n_heavy), "heavy_hi": hh[:n],
            "heavy_lo": hl[:n], "positions": int(res.positions), "seconds": secs}


def contigs(table: dict, k: int, forward_only: bool = False) -> list[str]:
    """Contigs of the UU k-mers of a table (as returned by run(); non-UU records are ignored),
    sorted (see orc_contigs in kmer_oracle.cpp for what a contig is)."""
    m = uu_mask(table)
    hi = np.ascontiguousarray(table["key_hi"][m], dtype=np.uint64)
    lo = np.ascontiguousarray(table["key_lo"][m], dtype=np.uint64)
    cl = np.ascontiguousarray(table["cls_l"][m], dtype=np.uint8)
    cr = np.ascontiguousarray(table["cls_r"][m], dtype=np.uint8)
    n = ctypes.c_int64()
    L = lib()
    h = L.orc_contigs(hi.ctypes.data, lo.ctypes.data, cl.ctypes.data, cr.ctypes.data, hi.size, k,
                      1 if forward_only else 0, ctypes.byref(n))
    if not h:
        raise ValueError("oracle contig generation failed")
    try:
        total = L.orc_contigs_bases(h)
        seq = np.zeros(max(total, 1), np.uint8)
        off = np.zeros(n.value + 1, np.int64)
        L.orc_contigs_fetch(h, seq.ctypes.data, off.ctypes.data)
    finally:
        L.orc_contigs_free(h)
    b = seq.tobytes()
    return [b[off[i]:off[i + 1]].decode() for i in range(n.value)]
