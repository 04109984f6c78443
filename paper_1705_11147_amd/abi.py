"""ctypes binding of include/hm_kmer.h (argument marshalling only).

Every entry point of the C ABI is exposed under its own name.  The library
must have been built (``__graft_entry__.build()`` or ``_build.build()``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

from . import _build

HM_OK = 0
HM_EINVAL = -1
HM_ECAPACITY = -2
HM_EHIP = -3
HM_EOUTPUT = -4
HM_EOVERFLOW = -5
HM_ETIMEOUT = -6

HM_ST_TABLE_FULL = 1
HM_ST_LIST_FULL = 2
HM_ST_OVERFLOW = 4
HM_ST_OUTPUT_FULL = 8
HM_ST_TIMEOUT = 16
HM_ST_DUPLICATE = 32
HM_ST_CLASSIFIED = 64
HM_ST_STREAM_FULL = 128

HM_FORWARD_ONLY = 1
HM_BLOOM_BYPASS = 2
HM_CHECKED = 4
HM_BLOOM_IN_TABLE = 8

HM_EXPORT_UU_ONLY = 1
HM_EXPORT_ALL = 2
HM_EXPORT_CLASSIFY = 4
HM_EXPORT_SORTED = 8
HM_MAX_HEAVY = 256
HM_EXPORT_STATIC_MAX_RECORDS = 1 << 18

HM_N_BIN_STATS = 6
HM_BINS_COUNTED = 1
BIN_STAT_NAMES = ("records", "spilled_bins", "spilled", "deferred", "keys", "kept")

HM_CLS_FORK = 4
HM_CLS_X = 5
HM_SLOT_BYTES = 64

u64p = ctypes.c_void_p  # device pointers travel as plain addresses


class Reads(ctypes.Structure):
    _fields_ = [("bases2", u64p), ("nmask", u64p), ("hqmask", u64p), ("read_off", u64p),
                ("n_reads", ctypes.c_int64), ("n_bases", ctypes.c_int64), ("read_len", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("min_depth", ctypes.c_uint32), ("ext_min", ctypes.c_uint32),
                ("n_owners", ctypes.c_uint32), ("owner", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


class Table(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("max_probe", ctypes.c_uint32),
                ("k", ctypes.c_int32), ("status", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("heavy", ctypes.c_void_p), ("n_heavy", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


STAT_NAMES = ["occurrences", "hit_first_lookup", "bloom_tests", "deferred", "probe_slots", "p2_entries",
              "p2_found", "cas_attempts", "wide_counts", "heavy_local", "probe_lines"]


class Bloom(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("n_words", ctypes.c_uint64), ("n_hash", ctypes.c_uint32)]


class List(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("ext", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("count", ctypes.c_void_p), ("present", ctypes.c_void_p), ("present_words", ctypes.c_uint64),
                ("present_hash", ctypes.c_uint32)]


class Export(ctypes.Structure):
    _fields_ = [("key_hi", ctypes.c_void_p), ("key_lo", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("tl", ctypes.c_void_p), ("tr", ctypes.c_void_p), ("cls_l", ctypes.c_void_p),
                ("cls_r", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("n_out", ctypes.c_void_p),
                ("digest", ctypes.c_void_p), ("min_depth", ctypes.c_uint32), ("ext_min", ctypes.c_uint32),
                ("sort_work", ctypes.c_void_p), ("sort_work_bytes", ctypes.c_uint64)]


class Card(ctypes.Structure):
    _fields_ = [("registers", ctypes.c_void_p), ("hll_p", ctypes.c_int32), ("sample_log2", ctypes.c_uint32),
                ("heavy_log2", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("positions", ctypes.c_void_p),
                ("sample", Table), ("heavy", Table)]


class CardSummary(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("sampled_distinct", ctypes.c_uint64),
                ("sampled_kept", ctypes.c_uint64), ("n_heavy", ctypes.c_uint64), ("positions", ctypes.c_uint64)]


class Occ(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("ext", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("count", ctypes.c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("recs", ctypes.c_void_p), ("tmp", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("group_bits", ctypes.c_uint32), ("bin_bits", ctypes.c_uint32), ("scratch", ctypes.c_void_p),
                ("bin_start", ctypes.c_void_p), ("status", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


class Contigs(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_void_p), ("seq_capacity", ctypes.c_uint64), ("off", ctypes.c_void_p),
                ("off_capacity", ctypes.c_uint64), ("counts", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_uint64)]


class BatchSet(ctypes.Structure):
    _fields_ = [("ascii", ctypes.c_void_p), ("qual", ctypes.c_void_p), ("n_reads", ctypes.c_int64),
                ("read_len", ctypes.c_int32), ("bases2", ctypes.c_void_p), ("nmask", ctypes.c_void_p),
                ("hqmask", ctypes.c_void_p), ("table", Table), ("bloom", Bloom), ("list", List), ("out", Export)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("tile_bases", ctypes.c_int32), ("list_per_item", ctypes.c_int32),
                ("slots_per_item", ctypes.c_int32), ("set_major", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("work", ctypes.c_void_p), ("n_sets", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("n_items", ctypes.c_int64), ("n_regions", ctypes.c_int64), ("pack_words", ctypes.c_int64),
                ("k", ctypes.c_int32), ("reserved", ctypes.c_int32)]


P = ctypes.POINTER
vp = ctypes.c_void_p
SIGNATURES = {
    "hm_abi_version": ([], ctypes.c_int),
    "hm_last_error": ([], ctypes.c_char_p),
    "hm_bases2_words": ([ctypes.c_int64], ctypes.c_uint64),
    "hm_mask_words": ([ctypes.c_int64], ctypes.c_uint64),
    "hm_table_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_bloom_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_list_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_export_sort_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_check_params": ([P(Params)], ctypes.c_int),
    "hm_table_init": ([P(Table), vp], ctypes.c_int),
    "hm_bloom_init": ([P(Bloom), vp], ctypes.c_int),
    "hm_list_init": ([P(List), vp], ctypes.c_int),
    "hm_status": ([P(Table), vp], ctypes.c_int),
    "hm_status_code": ([ctypes.c_uint32], ctypes.c_int),
    "hm_pack_reads": ([vp, vp, ctypes.c_int64, ctypes.c_uint8, ctypes.c_uint8, vp, vp, vp, vp], ctypes.c_int),
    "hm_bloom_insert": ([P(Reads), P(Params), P(Bloom), P(Table), P(List), vp], ctypes.c_int),
    "hm_kmer_count": ([P(Reads), P(Params), P(Table), P(List), vp], ctypes.c_int),
    "hm_classify_ext": ([P(Params), P(Table), vp], ctypes.c_int),
    "hm_export_table": ([P(Table), ctypes.c_uint32, P(Export), vp], ctypes.c_int),
    "hm_export_table_static": ([P(Table), ctypes.c_uint32, P(Export), vp], ctypes.c_int),
    "hm_card_init": ([P(Card), vp], ctypes.c_int),
    "hm_cardinality": ([P(Reads), P(Params), P(Card), vp], ctypes.c_int),
    "hm_card_summary": ([P(Card), ctypes.c_uint32, ctypes.c_uint32, vp, ctypes.c_uint64, vp, vp], ctypes.c_int),
    "hm_occ_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_occ_init": ([P(Occ), vp], ctypes.c_int),
    "hm_cardinality_occ": ([P(Reads), P(Params), P(Card), P(Occ), vp], ctypes.c_int),
    "hm_bloom_insert_occ": ([P(Occ), P(Params), P(Bloom), P(Table), P(List), vp], ctypes.c_int),
    "hm_bins_scratch_bytes": ([ctypes.c_uint32, ctypes.c_uint32], ctypes.c_size_t),
    "hm_bins_capacity": ([ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32], ctypes.c_uint64),
    "hm_bin_kmers": ([P(Reads), P(Params), P(Bins), ctypes.c_uint32, vp], ctypes.c_int),
    "hm_cardinality_bins": ([P(Reads), P(Params), P(Card), P(Bins), vp], ctypes.c_int),
    "hm_bin_occ": ([P(Occ), P(Params), P(Bins), vp], ctypes.c_int),
    "hm_count_bins": ([P(Bins), P(Params), ctypes.c_uint32, P(Export), P(Occ), vp], ctypes.c_int),
    "hm_export_merge": ([P(Export), P(Export), vp, vp], ctypes.c_int),
    "hm_contigs_work_bytes": ([ctypes.c_uint64], ctypes.c_size_t),
    "hm_contigs": ([P(Export), ctypes.c_int32, ctypes.c_uint32, P(Contigs), vp], ctypes.c_int),
    "hm_batch_work_bytes": ([ctypes.c_int32], ctypes.c_size_t),
    "hm_batch_prepare": ([P(BatchSet), ctypes.c_int32, P(Params), ctypes.c_uint8, ctypes.c_uint8, ctypes.c_uint32,
                          P(BatchTuning), vp, ctypes.c_size_t, P(BatchPlan), vp], ctypes.c_int),
    "hm_batch_launch": ([P(BatchPlan), vp], ctypes.c_int),
    "hm_random_access": ([vp, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, vp, vp],
                         ctypes.c_int),
}

HM_RA_LOAD = 0
HM_RA_LOAD_COHERENT = 1
HM_RA_ATOMIC_ADD = 2
HM_RA_ATOMIC_OR_RET = 3
HM_RA_LINE_RMW = 4
HM_RA_COPY = 5
HM_RA_PROBE_CAS = 6
HM_RA_SERIAL = 0x100

_LIB = None


class HmError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__("%s failed (%d): %s" % (what, code, msg))
        self.code = code


def lib(path: str | None = None):
    """Load libhm_kmer.so (built in-tree).  Raises if it is missing."""
    global _LIB
    if _LIB is None:
        so = path or _build.SO
        if not os.path.exists(so):
            raise RuntimeError("libhm_kmer.so is not built (%s); run __graft_entry__.build()" % so)
        L = ctypes.CDLL(so)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def last_error() -> str:
    return lib().hm_last_error().decode(errors="replace")


def check(rc: int, what: str) -> int:
    if rc != HM_OK:
        raise HmError(rc, what, last_error())
    return rc


def call(name: str, *args) -> int:
    """Call entry point `name`; raise HmError on a non-zero return."""
    return check(getattr(lib(), name)(*args), name)
