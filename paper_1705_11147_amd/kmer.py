"""k-mer analysis on the GPU through the C ABI.

PyTorch owns device memory and streams; every step of the path runs in the
HIP kernels of libhm_kmer.so (see include/hm_kmer.h).  The objects here only
allocate buffers, fill the ABI structs and call the entry points in order:

    hm_pack_reads -> hm_table_init / hm_bloom_init / hm_list_init
    -> hm_bloom_insert (per read batch) -> hm_kmer_count
    -> hm_classify_ext -> hm_export_table
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import abi

DEFAULT_SEED = 0x5DEECE66D


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def next_pow2(x: int) -> int:
    x = max(1, int(x))
    return 1 << (x - 1).bit_length()


def list_slack(pass1_launches: int = 1, device=None) -> int:
    """First-occurrence list entries a pass-1 launch can leave unused: every
    wave reserves list space in chunks of 256 entries and may strand up to
    255 at its end (8 blocks of 4 waves per CU)."""
    cus = torch.cuda.get_device_properties(device or torch.cuda.current_device()).multi_processor_count
    return int(pass1_launches) * cus * 8 * 4 * 255


def _empty_u64(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.int64, device=device)


def _new(n: int, dtype, device, alloc=None, zero: bool = False) -> torch.Tensor:
    """A 1-D tensor of max(n, 1) elements: from `alloc` (an object with empty(n, dtype), such as
    arena.Slab) when given, else from PyTorch's allocator on `device`.  zero: cleared on the
    current stream."""
    n = max(int(n), 1)
    t = torch.empty(n, dtype=dtype, device=device) if alloc is None else alloc.empty(n, dtype)
    return t.zero_() if zero else t


def _to_device(a: np.ndarray, device, alloc=None) -> torch.Tensor:
    """Copy a host array to a new device tensor: through pinned memory, asynchronously on the
    current stream, for a device; a plain copy for the CPU."""
    src = torch.from_numpy(np.ascontiguousarray(a))
    t = _new(src.numel(), src.dtype, device, alloc)[:src.numel()]
    if t.is_cuda:
        t.copy_(src.pin_memory(), non_blocking=True)
    else:
        t.copy_(src)
    return t


def tensor_bytes(n: int, itemsize: int) -> int:
    """Bytes a tensor of max(n, 1) elements takes in an arena slab (256-byte aligned)."""
    return (max(int(n), 1) * itemsize + 255) // 256 * 256


def packed_bytes(n_bases: int) -> int:
    """Bytes of the packed form of n_bases bases (hm_pack_reads' outputs) in an arena slab."""
    L = abi.lib()
    return tensor_bytes(L.hm_bases2_words(n_bases), 8) + 2 * tensor_bytes(L.hm_mask_words(n_bases), 8)


def new_packed(n_bases: int, device, alloc=None) -> "Packed":
    """Output buffers for pack_reads(out=...) of n_bases bases."""
    L = abi.lib()
    n_b2, n_m = int(L.hm_bases2_words(n_bases)), int(L.hm_mask_words(n_bases))
    return Packed(_new(n_b2, torch.int64, device, alloc), _new(n_m, torch.int64, device, alloc),
                  _new(n_m, torch.int64, device, alloc), None, 0, n_bases, 0)


def fetch_async(tensors, stream=None) -> list:
    """Queue copies of small device tensors into pinned host tensors on `stream` and return
    the host tensors.  They hold the values once the stream has passed this point (for
    instance once an event recorded after this call has completed): a host thread that
    serves many streams reads results without blocking on any of them."""
    st = stream if stream is not None else torch.cuda.current_stream()
    out = []
    with torch.cuda.stream(st):
        for t in tensors:
            h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
            h.copy_(t, non_blocking=True)
            out.append(h)
    return out


@dataclass
class Packed:
    """Packed reads resident on the device (layout: include/hm_kmer.h, hm_reads_t)."""
    bases2: torch.Tensor
    nmask: torch.Tensor
    hqmask: torch.Tensor
    read_off: torch.Tensor | None
    n_reads: int
    n_bases: int
    read_len: int

    def struct(self) -> abi.Reads:
        return abi.Reads(self.bases2.data_ptr(), self.nmask.data_ptr(), self.hqmask.data_ptr(),
                         self.read_off.data_ptr() if self.read_off is not None else None,
                         self.n_reads, self.n_bases, self.read_len)

    def positions(self, k: int) -> int:
        """Window count (upper bound of valid k-mer positions)."""
        if self.read_off is None:
            return self.n_reads * max(0, self.read_len - k + 1)
        lens = (self.read_off[1:] - self.read_off[:-1]).clamp(min=0)
        return int((lens - k + 1).clamp(min=0).sum().item())


def pack_reads(ascii: torch.Tensor, qual: torch.Tensor, read_len: int | None = None,
               read_off: torch.Tensor | None = None, qcut: int = 20, qual_offset: int = 0, stream=None,
               out: Packed | None = None) -> Packed:
    """hm_pack_reads on device-resident uint8 ascii/qual (same length)."""
    if ascii.dtype != torch.uint8 or qual.dtype != torch.uint8 or not ascii.is_cuda or not qual.is_cuda:
        raise TypeError("ascii and qual must be uint8 device tensors")
    n_bases = ascii.numel()
    if qual.numel() != n_bases:
        raise ValueError("ascii and qual differ in length")
    L = abi.lib()
    n_b2 = int(L.hm_bases2_words(n_bases))
    n_m = int(L.hm_mask_words(n_bases))
    if read_off is None:
        if not read_len:
            raise ValueError("give read_len or read_off")
        n_reads = n_bases // read_len
    else:
        read_off = read_off.to(device=ascii.device, dtype=torch.int64).contiguous()
        n_reads = read_off.numel() - 1
        read_len = 0
    if out is None or out.bases2.numel() < n_b2:
        out = Packed(_empty_u64(n_b2, ascii.device), _empty_u64(n_m, ascii.device), _empty_u64(n_m, ascii.device),
                     read_off, n_reads, n_bases, read_len or 0)
    else:
        out = Packed(out.bases2, out.nmask, out.hqmask, read_off, n_reads, n_bases, read_len or 0)
    abi.call("hm_pack_reads", ascii.data_ptr() if n_bases else None, qual.data_ptr() if n_bases else None, n_bases,
             qual_offset, qcut, out.bases2.data_ptr(), out.nmask.data_ptr(), out.hqmask.data_ptr(), _stream(stream))
    return out


class OccStream:
    """Owned-occurrence stream (hm_occ_t, 17 bytes per entry): written by the
    cardinality pass (CardSketch.update(..., occ=stream)), read by pass 1
    (KmerCounter.insert_occ) in place of the reads, for the sharded shape
    where an owner keeps a small share of all windows."""

    def __init__(self, capacity: int, device="cuda"):
        self.capacity = int(capacity)
        self.device = torch.device(device)
        n = max(self.capacity, 1)
        self.keys = torch.empty(2 * n, dtype=torch.int64, device=self.device)
        self.ext = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.count = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.occ = abi.Occ(self.keys.data_ptr(), self.ext.data_ptr(), self.capacity, self.count.data_ptr())

    @staticmethod
    def slack(launches: int = 1, device=None) -> int:
        """Entries a cardinality launch can leave as holes: every wave (4 per workgroup, 4 workgroups
        per CU) may leave up to 1023 of its last 1024-entry chunk unused."""
        cus = torch.cuda.get_device_properties(device or torch.cuda.current_device()).multi_processor_count
        return int(launches) * cus * 16 * 1023

    @classmethod
    def for_windows(cls, windows: int, n_owners: int, launches: int, device="cuda") -> "OccStream":
        """A stream for the owned share of `windows` windows: the expected share plus 2% and the
        hole slack (an overflow is reported and the pass rerun with a larger stream)."""
        share = int(windows / max(n_owners, 1) * 1.02) + 4096
        return cls(min(share, windows) + cls.slack(launches, device), device=device)

    @classmethod
    def view(cls, keys: torch.Tensor, ext: torch.Tensor, capacity: int, count: torch.Tensor) -> "OccStream":
        """A stream over existing buffers (2 * capacity int64 key words, capacity ext bytes, one
        int64 counter), e.g. the spill stream of BinnedCounter."""
        o = cls.__new__(cls)
        o.capacity, o.device = int(capacity), keys.device
        o.keys, o.ext, o.count = keys, ext, count
        o.occ = abi.Occ(keys.data_ptr(), ext.data_ptr(), o.capacity, count.data_ptr())
        return o

    def reset(self, stream=None):
        abi.call("hm_occ_init", ctypes.byref(self.occ), _stream(stream))

    def entries(self) -> int:
        """Entries reserved so far, holes included (synchronizes)."""
        return int(self.count.item())

    def overflowed(self) -> bool:
        return self.entries() > self.capacity


class Records:
    """Device export buffer (structure of arrays)."""

    def __init__(self, capacity: int, device="cuda", alloc=None):
        """alloc: take the buffers from this allocator (see _new) instead of PyTorch's."""
        self.capacity = int(capacity)
        n = max(self.capacity, 1)
        self.key_hi = _new(n, torch.int64, device, alloc)
        self.key_lo = _new(n, torch.int64, device, alloc)
        self.count = _new(n, torch.int32, device, alloc)
        self.tl = _new(n * 4, torch.int32, device, alloc)
        self.tr = _new(n * 4, torch.int32, device, alloc)
        self.cls_l = _new(n, torch.uint8, device, alloc)
        self.cls_r = _new(n, torch.uint8, device, alloc)
        self.n_out = _new(1, torch.int64, device, alloc, zero=True)
        self.digest = _new(2, torch.int64, device, alloc, zero=True)
        self.device = device
        self.sort_work = None

    @staticmethod
    def bytes_for(capacity: int) -> int:
        """Bytes the buffers of Records(capacity, alloc=slab) take in an arena slab."""
        n = max(int(capacity), 1)
        return (2 * tensor_bytes(n, 8) + tensor_bytes(n, 4) + 2 * tensor_bytes(4 * n, 4) + 2 * tensor_bytes(n, 1)
                + tensor_bytes(1, 8) + tensor_bytes(2, 8))

    def sort_scratch(self) -> tuple[int, int]:
        """(pointer, bytes) of the scratch a key-ordered export needs, allocated on first use."""
        need = int(abi.lib().hm_export_sort_bytes(self.capacity))
        if self.sort_work is None:
            self.sort_work = torch.empty(need // 8 + 64, dtype=torch.int64, device=self.device)
        base = self.sort_work.data_ptr()
        ptr = (base + 255) // 256 * 256
        return ptr, self.sort_work.numel() * 8 - (ptr - base)

    def struct(self, digest: bool = True, min_depth: int = 0, ext_min: int = 0, sort: bool = False) -> abi.Export:
        work, work_bytes = self.sort_scratch() if sort else (None, 0)
        return abi.Export(self.key_hi.data_ptr(), self.key_lo.data_ptr(), self.count.data_ptr(), self.tl.data_ptr(),
                          self.tr.data_ptr(), self.cls_l.data_ptr(), self.cls_r.data_ptr(), self.capacity,
                          self.n_out.data_ptr(), self.digest.data_ptr() if digest else None, min_depth, ext_min,
                          work, work_bytes)

    def to_numpy(self, n: int | None = None, sort: bool = True) -> dict:
        """Copy the first n records to the host (sorted by key when `sort`)."""
        n = int(self.n_out.item()) if n is None else n
        n = min(n, self.capacity)
        out = {
            "key_hi": self.key_hi[:n].cpu().numpy().view(np.uint64),
            "key_lo": self.key_lo[:n].cpu().numpy().view(np.uint64),
            "count": self.count[:n].cpu().numpy().view(np.uint32),
            "tl": self.tl[:4 * n].cpu().numpy().view(np.uint32).reshape(n, 4),
            "tr": self.tr[:4 * n].cpu().numpy().view(np.uint32).reshape(n, 4),
            "cls_l": self.cls_l[:n].cpu().numpy(),
            "cls_r": self.cls_r[:n].cpu().numpy(),
        }
        if sort:
            order = np.lexsort((out["key_lo"], out["key_hi"]))
            out = {key: v[order] for key, v in out.items()}
        return out

    def digest_words(self, fetched: tuple | None = None) -> tuple[int, int]:
        """The order-free digest; from the host copies fetch_summary() queued, if given."""
        d = (fetched[1] if fetched is not None else self.digest.cpu()).numpy().view(np.uint64)
        return int(d[0]), int(d[1])

    def fetch_summary(self, stream=None) -> tuple:
        """Queue copies of the record count and the digest into pinned host memory (see
        fetch_async): (n_out, digest) host tensors."""
        return tuple(fetch_async([self.n_out, self.digest], stream))

    @classmethod
    def from_numpy(cls, t: dict, device="cuda") -> "Records":
        """A device buffer holding host records (keys and classes; counters zero)."""
        n = len(t["key_hi"])
        r = cls(n, device=device)
        if n:
            r.key_hi[:n] = torch.from_numpy(np.ascontiguousarray(t["key_hi"], np.uint64).view(np.int64)).to(device)
            r.key_lo[:n] = torch.from_numpy(np.ascontiguousarray(t["key_lo"], np.uint64).view(np.int64)).to(device)
            r.cls_l[:n] = torch.from_numpy(np.ascontiguousarray(t["cls_l"], np.uint8)).to(device)
            r.cls_r[:n] = torch.from_numpy(np.ascontiguousarray(t["cls_r"], np.uint8)).to(device)
        r.count.zero_()
        r.tl.zero_()
        r.tr.zero_()
        r.n_out.fill_(n)
        return r


class ContigSet:
    """Contigs of the UU records of an export buffer (hm_contigs).

    capacity: records of the input buffers it serves; seq_capacity and
    off_capacity bound the bases and contigs (defaults: two bases per record
    plus one k-mer per 64 records, and one contig per 16 records); run()
    grows them when the device reports they were too small."""

    def __init__(self, capacity: int, k: int, seq_capacity: int | None = None, off_capacity: int | None = None,
                 device="cuda"):
        self.capacity, self.k, self.device = int(capacity), int(k), device
        need = int(abi.lib().hm_contigs_work_bytes(self.capacity))
        if need == 0:
            raise ValueError("contig generation takes fewer than 2^29 records")
        self.work = torch.empty(need // 8 + 64, dtype=torch.int64, device=device)
        self.counts = torch.zeros(2, dtype=torch.int64, device=device)
        self.status_buf = torch.zeros(1, dtype=torch.int32, device=device)
        self._alloc(seq_capacity if seq_capacity is not None else 2 * self.capacity + self.k * (self.capacity // 64 + 16),
                    off_capacity if off_capacity is not None else self.capacity // 16 + 1024)

    def _alloc(self, seq_capacity: int, off_capacity: int):
        self.seq_capacity, self.off_capacity = int(seq_capacity), int(off_capacity)
        self.seq = torch.empty(max(self.seq_capacity, 1), dtype=torch.uint8, device=self.device)
        self.off = torch.empty(self.off_capacity + 1, dtype=torch.int64, device=self.device)

    def struct(self) -> abi.Contigs:
        base = self.work.data_ptr()
        ptr = (base + 255) // 256 * 256
        return abi.Contigs(self.seq.data_ptr(), self.seq_capacity, self.off.data_ptr(), self.off_capacity,
                           self.counts.data_ptr(), self.status_buf.data_ptr(), ptr,
                           self.work.numel() * 8 - (ptr - base))

    def launch(self, records: Records, forward_only: bool = False, stream=None):
        """Queue the generation on the stream (no synchronization)."""
        if records.capacity > self.capacity:
            raise ValueError("input buffer holds %d records, set sized for %d" % (records.capacity, self.capacity))
        ex = records.struct(digest=False)
        cs = self.struct()
        abi.call("hm_contigs", ctypes.byref(ex), self.k, abi.HM_FORWARD_ONLY if forward_only else 0,
                 ctypes.byref(cs), _stream(stream))

    def run(self, records: Records, forward_only: bool = False, stream=None, retries: int = 2) -> int:
        """Generate, growing the outputs if they were too small; returns the status word."""
        for _ in range(retries + 1):
            self.launch(records, forward_only, stream)
            st = int(self.status_buf.item())
            if not st & abi.HM_ST_OUTPUT_FULL:
                return st
            nc, nb = (int(x) for x in self.counts.cpu().numpy())
            self._alloc(max(nb, self.seq_capacity), max(nc, self.off_capacity))
        return st

    def to_list(self, sort: bool = True) -> list[str]:
        nc, nb = (int(x) for x in self.counts.cpu().numpy())
        off = self.off[:nc + 1].cpu().numpy()
        b = self.seq[:nb].cpu().numpy().tobytes()
        out = [b[off[i]:off[i + 1]].decode() for i in range(nc)]
        return sorted(out) if sort else out


def contigs(records: Records, k: int, forward_only: bool = False, device=None) -> list[str]:
    """Sorted contigs of the UU records in an export buffer."""
    cs = ContigSet(records.capacity, k, device=device or records.device)
    st = cs.run(records, forward_only)
    if st:
        raise abi.HmError(abi.HM_EOUTPUT if st & abi.HM_ST_OUTPUT_FULL else abi.HM_EINVAL, "hm_contigs",
                          "status 0x%x" % st)
    return cs.to_list()


class KmerCounter:
    """One count table with its Bloom filter and first-occurrence list.

    capacity:       table slots (power of two, 64 bytes each)
    bloom_words:    Bloom filter size in 64-bit words (power of two); n_hash bits per key
    list_capacity:  first-occurrence list entries (17 bytes each): at most one per
                    distinct k-mer, plus list_slack() per pass-1 launch
    bloom_in_table: keep the filter in the table (abi.HM_BLOOM_IN_TABLE: one 32-bit word per
                    slot, tested on the line the probe has read); the table then gets at least
                    2 * bloom_words slots, so the filter has the bits asked for.  Otherwise a
                    separate filter of bloom_words words.
    """

    def __init__(self, k: int, capacity: int, bloom_words: int, list_capacity: int, n_hash: int = 4,
                 min_depth: int = 2, ext_min: int | None = None, n_owners: int = 1, owner: int = 0, flags: int = 0,
                 seed: int = DEFAULT_SEED, max_probe: int = 0, present_filter: bool = True, heavy=None,
                 bloom_in_table: bool = True, device="cuda", alloc=None):
        """heavy: optional heavy-hitter keys, an (n, 2) array of (key_hi, key_lo) or a CardResult;
        pass 1 counts them in workgroup-local memory (at most abi.HM_MAX_HEAVY).  alloc: take the
        buffers from this allocator (see _new) instead of PyTorch's.  The constructor's clears and
        the copy of the heavy keys are queued on the current stream."""
        self.device = torch.device(device)
        self.bypass = bool(flags & abi.HM_BLOOM_BYPASS) or min_depth == 1
        self.bloom_in_table = (bloom_in_table or bool(flags & abi.HM_BLOOM_IN_TABLE)) and not self.bypass
        flags = (flags | abi.HM_BLOOM_IN_TABLE) if self.bloom_in_table else (flags & ~abi.HM_BLOOM_IN_TABLE)
        self.params = abi.Params(k, min_depth, min_depth if ext_min is None else ext_min, n_owners, owner, flags,
                                 seed & (2 ** 64 - 1))
        abi.call("hm_check_params", ctypes.byref(self.params))
        if self.bloom_in_table:  # 32 filter bits per slot: at least the bits of bloom_words words
            capacity = max(capacity, 2 * int(bloom_words))
        self.capacity = next_pow2(capacity)
        self.slots = _new(self.capacity * abi.HM_SLOT_BYTES // 8, torch.int64, self.device, alloc)
        self.status_buf = _new(1, torch.int32, self.device, alloc, zero=True)
        self.stats_buf = _new(len(abi.STAT_NAMES), torch.int64, self.device, alloc, zero=True)
        if isinstance(heavy, CardResult):  # any subset of the heavy hitters gives the same counts
            n = min(len(heavy.heavy_hi), abi.HM_MAX_HEAVY)
            heavy = np.stack([heavy.heavy_hi[:n], heavy.heavy_lo[:n]], axis=1) if n else None
        hk = np.zeros((0, 2), np.uint64) if heavy is None else np.asarray(heavy, dtype=np.uint64).reshape(-1, 2)
        if len(hk) > abi.HM_MAX_HEAVY:
            raise ValueError("at most %d heavy keys" % abi.HM_MAX_HEAVY)
        self.heavy_keys = _to_device(hk.view(np.int64).reshape(-1), self.device, alloc) if len(hk) else None
        self.table = abi.Table(self.slots.data_ptr(), self.capacity, max_probe, k, self.status_buf.data_ptr(),
                               self.stats_buf.data_ptr(),
                               self.heavy_keys.data_ptr() if self.heavy_keys is not None else None, len(hk), 0)
        self.bloom_words = next_pow2(bloom_words) if not (self.bypass or self.bloom_in_table) else 1
        self.bloom_buf = _new(self.bloom_words, torch.int64, self.device, alloc)
        self.bloom = abi.Bloom(self.bloom_buf.data_ptr(), self.bloom_words, n_hash)
        self.list_capacity = int(list_capacity) if not self.bypass else 0
        lc = max(self.list_capacity, 1)
        self.list_keys = _new(2 * lc, torch.int64, self.device, alloc)
        self.list_ext = _new(lc, torch.uint8, self.device, alloc)
        self.list_count = _new(1, torch.int64, self.device, alloc, zero=True)
        # presence filter of inserted keys: about 8 bits per key at the table's design load
        self.present_words = 0 if (self.bypass or not present_filter) else next_pow2(max(64, self.capacity // 16))
        self.present_buf = _new(self.present_words, torch.int64, self.device, alloc)
        self.list = abi.List(self.list_keys.data_ptr(), self.list_ext.data_ptr(), self.list_capacity,
                             self.list_count.data_ptr(), self.present_buf.data_ptr() if self.present_words else None,
                             self.present_words, 3)

    @staticmethod
    def bytes_for(capacity: int, bloom_words: int, list_capacity: int, n_heavy: int = 0, min_depth: int = 2,
                  flags: int = 0, present_filter: bool = True, bloom_in_table: bool = True) -> int:
        """Bytes the buffers of KmerCounter(..., alloc=slab) take in an arena slab (the same
        sizing rules as the constructor)."""
        bypass = bool(flags & abi.HM_BLOOM_BYPASS) or min_depth == 1
        in_table = (bloom_in_table or bool(flags & abi.HM_BLOOM_IN_TABLE)) and not bypass
        if in_table:
            capacity = max(capacity, 2 * int(bloom_words))
        cap = next_pow2(capacity)
        words = next_pow2(bloom_words) if not (bypass or in_table) else 1
        lc = max(int(list_capacity) if not bypass else 0, 1)
        pw = 0 if (bypass or not present_filter) else next_pow2(max(64, cap // 16))
        return (tensor_bytes(cap * abi.HM_SLOT_BYTES // 8, 8) + tensor_bytes(1, 4)
                + tensor_bytes(len(abi.STAT_NAMES), 8) + (tensor_bytes(2 * n_heavy, 8) if n_heavy else 0)
                + tensor_bytes(words, 8) + tensor_bytes(2 * lc, 8) + tensor_bytes(lc, 1) + tensor_bytes(1, 8)
                + tensor_bytes(pw, 8))

    @property
    def k(self) -> int:
        return self.params.k

    def bytes(self) -> int:
        return (self.slots.numel() + self.bloom_buf.numel() + self.list_keys.numel() + self.present_buf.numel()) * 8 \
            + self.list_ext.numel()

    # ---- the steps, each one C-ABI call ----
    def reset(self, stream=None):
        s = _stream(stream)
        abi.call("hm_table_init", ctypes.byref(self.table), s)
        if not self.bypass:
            if not self.bloom_in_table:  # else hm_table_init cleared it
                abi.call("hm_bloom_init", ctypes.byref(self.bloom), s)
            abi.call("hm_list_init", ctypes.byref(self.list), s)

    def insert(self, packed: Packed, stream=None):
        r = packed.struct()
        abi.call("hm_bloom_insert", ctypes.byref(r), ctypes.byref(self.params),
                 None if self.bypass else ctypes.byref(self.bloom), ctypes.byref(self.table),
                 None if self.bypass else ctypes.byref(self.list), _stream(stream))

    def insert_occ(self, occ: "OccStream", stream=None):
        """Pass 1 over an owned-occurrence stream written by the cardinality pass."""
        abi.call("hm_bloom_insert_occ", ctypes.byref(occ.occ), ctypes.byref(self.params),
                 None if self.bypass else ctypes.byref(self.bloom), ctypes.byref(self.table),
                 None if self.bypass else ctypes.byref(self.list), _stream(stream))

    def count(self, stream=None):
        abi.call("hm_kmer_count", None, ctypes.byref(self.params), ctypes.byref(self.table),
                 None if self.bypass else ctypes.byref(self.list), _stream(stream))

    def classify(self, stream=None):
        abi.call("hm_classify_ext", ctypes.byref(self.params), ctypes.byref(self.table), _stream(stream))

    def export(self, out: Records, flags: int = 0, stream=None, digest: bool = True, static: bool = False):
        """hm_export_table; with abi.HM_EXPORT_CLASSIFY in flags the export
        classifies from the counters (no hm_classify_ext needed before).  static: the
        no-allocation variant hm_export_table_static (a key-ordered export's scratch is the
        library's own array; out.capacity <= abi.HM_EXPORT_STATIC_MAX_RECORDS)."""
        sort = bool(flags & abi.HM_EXPORT_SORTED) and not static
        e = out.struct(digest, self.params.min_depth, self.params.ext_min, sort=sort)
        abi.call("hm_export_table_static" if static else "hm_export_table", ctypes.byref(self.table), flags,
                 ctypes.byref(e), _stream(stream))

    def stats(self) -> dict:
        """Event counters of the counting passes (synchronizes)."""
        return dict(zip(abi.STAT_NAMES, (int(x) for x in self.stats_buf.cpu().numpy())))

    def status(self, stream=None) -> int:
        """Synchronize and return the table's status code (HM_OK or a negative code)."""
        return abi.lib().hm_status(ctypes.byref(self.table), _stream(stream))

    def fetch_status(self, stream=None) -> torch.Tensor:
        """Queue a copy of the status word into pinned host memory (see fetch_async);
        status_code() of it, once the stream has passed, is what status() returns."""
        return fetch_async([self.status_buf], stream)[0]

    @staticmethod
    def status_code(word: torch.Tensor) -> int:
        return abi.lib().hm_status_code(int(word[0]) & 0xFFFFFFFF)

    def run(self, batches, out: Records, flags: int = 0, stream=None, digest: bool = True, fused: bool = False):
        """reset -> pass 1 over every packed batch -> pass 2 -> classify -> export
        (all async).  fused: classify inside the export sweep instead."""
        self.reset(stream)
        for p in batches:
            self.insert(p, stream)
        self._finish(out, flags, stream, digest, fused)

    def run_occ(self, occ: OccStream, out: Records, flags: int = 0, stream=None, digest: bool = True,
                fused: bool = False):
        """As run(), with pass 1 over an owned-occurrence stream instead of the reads."""
        self.reset(stream)
        self.insert_occ(occ, stream)
        self._finish(out, flags, stream, digest, fused)

    def _finish(self, out: Records, flags: int, stream, digest: bool, fused: bool):
        self.count(stream)
        if fused:
            self.export(out, flags | abi.HM_EXPORT_CLASSIFY, stream, digest)
        else:
            self.classify(stream)
            self.export(out, flags, stream, digest)


@dataclass
class CardResult:
    """Summary of a cardinality pass (hm_card_summary), copied to the host."""
    estimate: float          # HyperLogLog estimate of distinct owned k-mers
    sampled_distinct: int    # keys in the distinct sample (1 in 2^sample_log2 keys)
    sampled_kept: int        # of those, keys with count >= min_depth
    n_heavy: int             # keys whose window-sample count reached heavy_min
    positions: int           # valid windows of owned keys
    hll_p: int
    sample_log2: int
    heavy_log2: int
    heavy_hi: np.ndarray
    heavy_lo: np.ndarray
    status: int              # HM_OK, or HM_ECAPACITY when a sample table filled up

    def distinct_hi(self, z: float = 4.0) -> float:
        """Upper bound on the distinct k-mers: z standard errors (1.04/sqrt(m)) above the estimate."""
        return self.estimate * (1.0 + z * 1.04 / (1 << self.hll_p) ** 0.5) + z

    def kept_hi(self, z: float = 4.0) -> float:
        """Upper bound on the k-mers that pass the depth filter: the sampled count plus z Poisson
        standard deviations, scaled by the sampling rate."""
        s = float(1 << self.sample_log2)
        return min((self.sampled_kept + z * self.sampled_kept ** 0.5 + z) * s, self.distinct_hi(z))


class CardSketch:
    """State of the cardinality pass (C ABI hm_card_*): HyperLogLog registers, the distinct-sample
    table and the window-sample table.  Sample rates default to about 2^18 sampled keys and
    windows for `positions_hint` windows, so a heavy hitter (heavy_min = 16 sampled windows) is
    a k-mer holding at least 2^-14 of all windows."""

    def __init__(self, k: int, positions_hint: int, hll_p: int = 14, sample_log2: int | None = None,
                 heavy_log2: int | None = None, n_owners: int = 1, owner: int = 0, forward_only: bool = False,
                 seed: int = DEFAULT_SEED, device="cuda", alloc=None):
        """alloc: take the buffers from this allocator (see _new) instead of PyTorch's."""
        self.device = torch.device(device)
        self.params = abi.Params(k, 2, 2, n_owners, owner, abi.HM_FORWARD_ONLY if forward_only else 0,
                                 seed & (2 ** 64 - 1))
        abi.call("hm_check_params", ctypes.byref(self.params))
        hint = max(int(positions_hint), 1)
        auto = max(0, hint.bit_length() - 18)
        self.hll_p = hll_p
        self.sample_log2 = auto if sample_log2 is None else sample_log2
        self.heavy_log2 = auto if heavy_log2 is None else heavy_log2
        self.registers = _new(1 << hll_p, torch.int32, self.device, alloc, zero=True)
        self.positions = _new(1, torch.int64, self.device, alloc, zero=True)
        self._tabs = []
        tables = []
        for log2 in (self.sample_log2, self.heavy_log2):
            cap = next_pow2(max(1024, 2 * (hint >> log2) + 256))
            slots = _new(cap * abi.HM_SLOT_BYTES // 8, torch.int64, self.device, alloc)
            status = _new(1, torch.int32, self.device, alloc, zero=True)
            self._tabs.append((slots, status))
            tables.append(abi.Table(slots.data_ptr(), cap, 0, k, status.data_ptr(), None))
        self.card = abi.Card(self.registers.data_ptr(), hll_p, self.sample_log2, self.heavy_log2, 0,
                             self.positions.data_ptr(), tables[0], tables[1])
        self.summary_buf = _new(5, torch.int64, self.device, alloc, zero=True)
        self.heavy_cap = 4096
        self.heavy_keys = _new(2 * self.heavy_cap, torch.int64, self.device, alloc, zero=True)

    @staticmethod
    def bytes_for(positions_hint: int, hll_p: int = 14, sample_log2: int | None = None,
                  heavy_log2: int | None = None) -> int:
        """Bytes the buffers of CardSketch(..., alloc=slab) take in an arena slab (default heavy_cap)."""
        hint = max(int(positions_hint), 1)
        auto = max(0, hint.bit_length() - 18)
        total = tensor_bytes(1 << hll_p, 4) + tensor_bytes(1, 8) + tensor_bytes(5, 8) + tensor_bytes(2 * 4096, 8)
        for log2 in (auto if sample_log2 is None else sample_log2, auto if heavy_log2 is None else heavy_log2):
            cap = next_pow2(max(1024, 2 * (hint >> log2) + 256))
            total += tensor_bytes(cap * abi.HM_SLOT_BYTES // 8, 8) + tensor_bytes(1, 4)
        return total

    def reset(self, stream=None):
        abi.call("hm_card_init", ctypes.byref(self.card), _stream(stream))

    def update(self, packed: Packed, stream=None, occ: OccStream | None = None, bins: "BinnedCounter | None" = None):
        """Add a batch of reads; with `occ`, also append its owned occurrences to that stream; with
        `bins`, also count the first partition level's histogram of those bins (then call
        bins.bin(packed, counted=True) next, with the same reads)."""
        r = packed.struct()
        if bins is not None:
            if occ is not None:
                raise ValueError("update: occ and bins are exclusive")
            abi.call("hm_cardinality_bins", ctypes.byref(r), ctypes.byref(self.params), ctypes.byref(self.card),
                     ctypes.byref(bins.bins), _stream(stream))
        elif occ is None:
            abi.call("hm_cardinality", ctypes.byref(r), ctypes.byref(self.params), ctypes.byref(self.card),
                     _stream(stream))
        else:
            abi.call("hm_cardinality_occ", ctypes.byref(r), ctypes.byref(self.params), ctypes.byref(self.card),
                     ctypes.byref(occ.occ), _stream(stream))

    def summarize(self, min_depth: int = 2, heavy_min: int = 16, heavy_cap: int | None = None, stream=None):
        """Launch hm_card_summary (asynchronous); result() reads it.  Up to heavy_cap heavy keys
        are kept (default 4096; a larger cap reallocates the key buffer)."""
        if heavy_cap is not None and heavy_cap != self.heavy_cap:
            self.heavy_cap = heavy_cap
            self.heavy_keys = torch.zeros(2 * max(heavy_cap, 1), dtype=torch.int64, device=self.device)
        abi.call("hm_card_summary", ctypes.byref(self.card), min_depth, heavy_min, self.heavy_keys.data_ptr(),
                 self.heavy_cap, self.summary_buf.data_ptr(), _stream(stream))

    def fetch(self, stream=None) -> list:
        """Queue copies of the summary hm_card_summary wrote (and of the sample tables' status
        words) into pinned host memory on the stream (see fetch_async); decode() them once the
        stream has passed."""
        return fetch_async([self.summary_buf, self.heavy_keys] + [status for _, status in self._tabs], stream)

    def decode(self, fetched: list) -> CardResult:
        raw = fetched[0].numpy()
        est = float(raw[:1].view(np.float64)[0])
        u = raw.view(np.uint64)
        n_heavy = int(u[3])
        hk = fetched[1].numpy()[: 2 * min(n_heavy, self.heavy_cap)].view(np.uint64).reshape(-1, 2)
        order = np.lexsort((hk[:, 1], hk[:, 0])) if len(hk) else np.zeros(0, np.int64)
        rc = abi.HM_OK
        for status in fetched[2:]:
            if int(status[0]) & abi.HM_ST_TABLE_FULL:
                rc = abi.HM_ECAPACITY
        return CardResult(est, int(u[1]), int(u[2]), n_heavy, int(u[4]), self.hll_p, self.sample_log2,
                          self.heavy_log2, hk[order, 0].copy(), hk[order, 1].copy(), rc)

    def result(self, stream=None) -> CardResult:
        """Synchronize the stream and return the summary."""
        fetched = self.fetch(stream)
        torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
        return self.decode(fetched)

    def run(self, batches, min_depth: int = 2, heavy_min: int = 16, heavy_cap: int | None = None,
            stream=None, occ: OccStream | None = None) -> CardResult:
        """The whole pass over `batches`; with `occ` (reset here) their owned occurrences are written to it."""
        self.reset(stream)
        if occ is not None:
            occ.reset(stream)
        for p in batches:
            self.update(p, stream, occ)
        self.summarize(min_depth, heavy_min, heavy_cap, stream)
        return self.result(stream)


def bloom_fp_rate(bits_per_key: float, n_hash: int, word_bits: int = 64) -> float:
    """False-positive rate of the single-word blocked Bloom filter (every key's n_hash bits in one
    word of word_bits bits: 64 for the separate filter, 32 for the filter in the table) at its
    final load: keys per word ~ Poisson(word_bits / bits_per_key)."""
    lam = word_bits / max(bits_per_key, 1e-9)
    # Poisson weights in log space over the mass around the mode (no underflow at any load)
    lo = max(0, int(lam - 12.0 * np.sqrt(lam)) - 8)
    j = np.arange(lo, int(lam + 12.0 * np.sqrt(lam)) + 64, dtype=np.float64)
    logp = j * np.log(lam) - lam - np.array([math.lgamma(x + 1.0) for x in j])
    # P(a new key's n_hash bits are all set | j keys in its word): the word has x bits set after
    # the j keys' n_hash * j uniform draws (occupancy of word_bits bins, one more draw at a time:
    # x stays with probability x / word_bits), and the n_hash test bits all fall among them with
    # probability (x / word_bits)^n_hash
    w = word_bits
    x = np.arange(w + 1, dtype=np.float64)
    hit = (x / w) ** n_hash
    occ = np.zeros(w + 1)
    occ[0] = 1.0
    cond = np.ones(len(j))
    for m in range(n_hash * (int(j[-1]) + 1)):
        if m % n_hash == 0 and m // n_hash >= lo:
            cond[m // n_hash - lo] = occ @ hit
            if occ[w] > 1.0 - 1e-15:  # every bit set from here on
                break
        nxt = occ * (x / w)
        nxt[1:] += occ[:-1] * ((w - x[:-1]) / w)
        occ = nxt
    return min(1.0, float(np.sum(np.exp(logp) * cond)))


def plan_sizes(card: CardResult, n_hash: int = 4, bloom_bits: float = 12.0, table_load: float = 0.5,
               pass1_launches: int = 1, device=None, bloom_in_table: bool = True) -> tuple[int, int, int]:
    """(table capacity, Bloom words, list capacity) from a cardinality pass, the way the paper
    sizes its Bloom filter from the HyperLogLog estimate: the filter gets `bloom_bits` bits per
    distinct k-mer (Bloom words: its size in 64-bit words); the table holds the kept k-mers plus
    the singletons the filter lets through, and with the filter in the table (32 bits per slot)
    at least the filter's bits; the first-occurrence list holds at most one entry per distinct
    k-mer plus the per-launch chunk slack."""
    d_hi = card.distinct_hi()
    kept_hi = card.kept_hi()
    bloom_words = next_pow2(max(64, int(d_hi * bloom_bits / 64)))
    if bloom_in_table:
        floor = max(1024, 2 * bloom_words)
        fp = bloom_fp_rate(floor * 32 / max(d_hi, 1.0), n_hash, word_bits=32)  # a bigger table only lowers it
        capacity = next_pow2(max(floor, int((kept_hi + fp * max(d_hi - kept_hi, 0.0)) / table_load)))
    else:
        fp = bloom_fp_rate(bloom_words * 64 / max(d_hi, 1.0), n_hash)
        capacity = next_pow2(max(1024, int((kept_hi + fp * max(d_hi - kept_hi, 0.0)) / table_load)))
    lcap = int(d_hi) + list_slack(pass1_launches, device)
    return capacity, bloom_words, lcap


BIN_SLOTS = 512       # local table of a bin (hm_count_bins spills a bin past 384 keys)
BIN_DEFER_CAP = 2048  # deferred occurrences a bin holds
MAX_GROUP_BITS = 10   # first partition level
MAX_BIN_BITS = 11     # second partition level (bins per group)


def plan_bins(distinct_hi: float, seen2_hi: float, bypass: bool = False) -> tuple[int, int]:
    """(group_bits, bin_bits) for the binned path: enough bins that a bin's distinct k-mers (its
    deferred occurrences, about one per distinct k-mer) stay near 900 of the 2048 its list holds,
    and the k-mers it inserts (those seen at least twice, or with the Bloom filter bypassed every
    distinct k-mer) near 192 of the 384 its table takes before the bin spills; at most 2^21 bins, and
    2^20 while that keeps a bin within 25% of those targets.
    The second level takes up to 11 bits and at least half, so that small inputs still spread
    over many first-level groups."""
    need = seen2_hi / 192.0 if not bypass else distinct_hi / 192.0
    need = max(1.0, need, distinct_hi / 900.0)
    total = min(MAX_GROUP_BITS + MAX_BIN_BITS, max(0, int(math.ceil(math.log2(need)))))
    # 2^10 first-level groups leave the first-level scatter one workgroup a CU (its LDS), so up to
    # 25% past the targets (about 240 keys a bin, far from the 384 that spill) 2^20 bins are faster
    if total == MAX_GROUP_BITS + MAX_BIN_BITS and need <= 1.25 * 2.0 ** (total - 1):
        total -= 1
    b = min(MAX_BIN_BITS, total, max(total - MAX_GROUP_BITS, (total + 3) // 2))
    return total - b, b


class BinnedCounter:
    """The binned path (hm_bin_kmers, hm_count_bins): the occurrences partitioned by key hash into
    bins small enough for a workgroup's local memory, each bin counted there with its own Bloom
    filter and table.  Bins that do not fit go to a spill stream (in the buffer the partition
    used as scratch) and are counted by the global-table path (KmerCounter.insert_occ), whose
    export is merged into the binned one.

    windows: the read set's windows, n_reads * (read_len - k + 1) (the buffers hold those plus the
    padding of the partition's ranges, abi hm_bins_capacity)."""

    def __init__(self, k: int, windows: int, group_bits: int, bin_bits: int, min_depth: int = 2,
                 ext_min: int | None = None, n_owners: int = 1, owner: int = 0, flags: int = 0,
                 seed: int = DEFAULT_SEED, device="cuda", alloc=None):
        self.device = torch.device(device)
        self.bypass = bool(flags & abi.HM_BLOOM_BYPASS) or min_depth == 1
        self.params = abi.Params(k, min_depth, min_depth if ext_min is None else ext_min, n_owners, owner,
                                 flags & ~abi.HM_BLOOM_IN_TABLE, seed & (2 ** 64 - 1))
        abi.call("hm_check_params", ctypes.byref(self.params))
        self.group_bits, self.bin_bits = int(group_bits), int(bin_bits)
        self.capacity = int(abi.lib().hm_bins_capacity(int(windows), self.group_bits, self.bin_bits))
        if self.capacity == 0:
            raise ValueError("group_bits must be at most %d and bin_bits at most %d" % (MAX_GROUP_BITS, MAX_BIN_BITS))
        self.n_bins = 1 << (self.group_bits + self.bin_bits)
        n = max(self.capacity, 1)
        self.recs = _new(2 * n, torch.int64, self.device, alloc)
        self.tmp = _new(2 * n, torch.int64, self.device, alloc)
        self.spill_ext = _new(n, torch.uint8, self.device, alloc)
        sb = abi.lib().hm_bins_scratch_bytes(self.group_bits, self.bin_bits)
        self.scratch = _new((sb + 7) // 8, torch.int64, self.device, alloc)
        self.bin_start = _new(self.n_bins + 1, torch.int64, self.device, alloc)
        self.status_buf = _new(1, torch.int32, self.device, alloc, zero=True)
        self.stats_buf = _new(abi.HM_N_BIN_STATS, torch.int64, self.device, alloc, zero=True)
        self.spill_count = _new(1, torch.int64, self.device, alloc, zero=True)
        self.bins = abi.Bins(self.recs.data_ptr(), self.tmp.data_ptr(), self.capacity, self.group_bits,
                             self.bin_bits, self.scratch.data_ptr(), self.bin_start.data_ptr(),
                             self.status_buf.data_ptr(), self.stats_buf.data_ptr())
        self.spill = OccStream.view(self.tmp, self.spill_ext, self.capacity, self.spill_count)
        self.fallback = None  # the KmerCounter of the last spilled run

    @property
    def k(self) -> int:
        return self.params.k

    def bin(self, packed: Packed, stream=None, counted: bool = False):
        """Partition the reads' windows into the bins; counted: CardSketch.update(packed, bins=self)
        has just counted the first level's histogram."""
        r = packed.struct()
        abi.call("hm_bin_kmers", ctypes.byref(r), ctypes.byref(self.params), ctypes.byref(self.bins),
                 abi.HM_BINS_COUNTED if counted else 0, _stream(stream))

    def bin_occ(self, occ: OccStream, stream=None):
        """Partition an owned-occurrence stream (CardSketch.update(..., occ=stream)) into the bins,
        in place of the reads: build the counter with windows = occ.capacity."""
        abi.call("hm_bin_occ", ctypes.byref(occ.occ), ctypes.byref(self.params), ctypes.byref(self.bins),
                 _stream(stream))

    def count(self, out: Records, flags: int = 0, stream=None, digest: bool = True):
        """hm_count_bins into `out` (flags: 0 or abi.HM_EXPORT_UU_ONLY); spilled bins are left in the
        spill stream (see finish)."""
        ex = out.struct(digest=digest)
        abi.call("hm_count_bins", ctypes.byref(self.bins), ctypes.byref(self.params), flags, ctypes.byref(ex),
                 ctypes.byref(self.spill.occ), _stream(stream))

    def spilled(self) -> int:
        """Records sent to the spill stream (synchronizes)."""
        return int(self.spill_count.item())

    def finish(self, out: Records, flags: int = 0, stream=None, digest: bool = True, distinct_per_record: float = 1.0,
               retries: int = 4) -> int:
        """Count the spill stream with the global-table path and merge its export into `out`
        (nothing to do when no bin spilled).  distinct_per_record bounds the distinct k-mers per
        spilled record for sizing the table (doubled and rerun on a capacity error).  Returns the
        spilled records."""
        n = self.spilled()
        if n == 0:
            return 0
        est = max(1024, int(n * min(1.0, distinct_per_record)) + 1)
        cap = next_pow2(2 * est)
        for _ in range(retries + 1):
            kc = KmerCounter(self.k, cap, 64, n + list_slack(1, self.device), min_depth=self.params.min_depth,
                             ext_min=self.params.ext_min, flags=self.params.flags, seed=self.params.seed,
                             device=self.device)
            out2 = Records(max(1, cap // 2), device=self.device)
            kc.reset(stream)
            kc.insert_occ(self.spill, stream)
            kc.count(stream)
            kc.export(out2, flags | abi.HM_EXPORT_CLASSIFY, stream, digest=digest)
            rc = kc.status(stream)
            if rc == abi.HM_ECAPACITY:
                cap *= 2
                continue
            abi.check(rc, "binned path: the spilled bins")
            ex2, ex = out2.struct(digest=digest), out.struct(digest=digest)
            abi.call("hm_export_merge", ctypes.byref(ex2), ctypes.byref(ex), self.status_buf.data_ptr(),
                     _stream(stream))
            self.fallback = kc
            return n
        raise abi.HmError(abi.HM_ECAPACITY, "binned path: the spilled bins", "still full after %d retries" % retries)

    def run(self, packed: Packed, out: Records, flags: int = 0, stream=None, digest: bool = True,
            distinct_per_record: float = 1.0) -> int:
        """The whole binned path over one read set; returns the spilled records."""
        self.bin(packed, stream)
        self.count(out, flags, stream, digest)
        return self.finish(out, flags, stream, digest, distinct_per_record)

    def stats(self) -> dict:
        v = self.stats_buf.cpu().numpy()
        return {name: int(x) for name, x in zip(abi.BIN_STAT_NAMES, v)}

    def status(self, stream=None) -> int:
        """Code of the bins' status word (synchronizes)."""
        (torch.cuda.current_stream(self.device) if stream is None else stream).synchronize()
        return abi.lib().hm_status_code(int(self.status_buf.item()) & 0xFFFFFFFF)

    def bin_sizes(self) -> np.ndarray:
        return np.diff(self.bin_start.cpu().numpy())


def analyze(ascii: np.ndarray, qual: np.ndarray, k: int, read_len: int | None = None,
            read_off: np.ndarray | None = None, qcut: int = 20, qual_offset: int = 0, min_depth: int = 2,
            ext_min: int | None = None, n_owners: int = 1, owner: int = 0, forward_only: bool = False,
            bypass: bool = False, checked: bool = False, export_flags: int = 0, capacity: int | None = None,
            bloom_words: int | None = None, n_hash: int = 4, list_capacity: int | None = None,
            seed: int = DEFAULT_SEED, max_probe: int = 0, device="cuda", retries: int = 4, fused: bool = False,
            present_filter: bool = True, sizing: str = "card", heavy: bool = True,
            bloom_in_table: bool = True, occ_stream: bool = False, occ_capacity: int | None = None,
            binned: bool = False, bin_bits: tuple[int, int] | None = None) -> dict:
    """Host arrays in, sorted host table out (the whole path on the GPU).

    Sizes not given are planned from a cardinality pass over the reads
    (sizing="card": HyperLogLog estimate and distinct sample, plan_sizes) or
    set to worst-case bounds from the number of windows (sizing="bound").  On
    a capacity error the table (or list) is doubled and the run repeated from
    scratch, which keeps the result exact.  heavy: count the heavy hitters the
    cardinality pass finds in workgroup-local memory (sizing="card" only).  bloom_in_table: the
    Bloom filter in the table's slots (KmerCounter) or a separate one.  occ_stream: the
    cardinality pass writes the owned occurrences to a stream (occ_capacity entries, default
    OccStream.for_windows; doubled and rerun on overflow) and pass 1 reads it instead of the
    reads (sizing="card" only).  binned: the binned path (BinnedCounter: fixed-length reads,
    k <= 61), with (group_bits, bin_bits) from plan_bins over a cardinality pass unless bin_bits
    is given; with occ_stream too, the bins are filled from the stream the cardinality pass writes
    (hm_bin_occ) instead of from the reads; its records are those of the table path."""
    dev = torch.device(device)
    a = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8)).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(qual, dtype=np.uint8)).to(dev)
    off = None if read_off is None else torch.from_numpy(np.ascontiguousarray(read_off, dtype=np.int64)).to(dev)
    packed = pack_reads(a, q, read_len=read_len, read_off=off, qcut=qcut, qual_offset=qual_offset)
    P = packed.positions(k)
    flags = (abi.HM_FORWARD_ONLY if forward_only else 0) | (abi.HM_BLOOM_BYPASS if bypass else 0) | \
        (abi.HM_CHECKED if checked else 0)
    if binned:
        occ = None
        if bin_bits is None or occ_stream:
            sk = CardSketch(k, P, n_owners=n_owners, owner=owner, forward_only=forward_only, seed=seed, device=dev)
            if occ_stream:  # the owned occurrences written by the cardinality pass, partitioned from there
                occ = OccStream(occ_capacity, device=dev) if occ_capacity is not None else \
                    OccStream.for_windows(P, n_owners, 1, device=dev)
                while True:
                    c2 = sk.run([packed], min_depth=2, occ=occ)
                    if not occ.overflowed():
                        break
                    occ = OccStream(2 * max(occ.capacity, occ.entries()), device=dev)
            else:
                c2 = sk.run([packed], min_depth=2)
            if bin_bits is None:
                bin_bits = plan_bins(c2.distinct_hi(), c2.kept_hi(), bypass or min_depth == 1)
            del sk
        bc = BinnedCounter(k, occ.capacity if occ is not None else P, bin_bits[0], bin_bits[1], min_depth=min_depth,
                           ext_min=ext_min, n_owners=n_owners, owner=owner, flags=flags, seed=seed, device=dev)
        out = Records(max(1024, P), device=dev)
        if occ is not None:
            bc.bin_occ(occ)
            bc.count(out, export_flags & abi.HM_EXPORT_UU_ONLY)
            spilled = bc.finish(out, export_flags & abi.HM_EXPORT_UU_ONLY)
        else:
            spilled = bc.run(packed, out, export_flags & abi.HM_EXPORT_UU_ONLY)
        abi.check(bc.status(), "binned k-mer analysis")
        res = out.to_numpy(sort=True)
        res["digest"] = out.digest_words()
        res["positions"] = P
        res["bin_stats"] = bc.stats()
        res["spilled"] = spilled
        res["bin_bits"] = tuple(bin_bits)
        return res
    card = None
    occ = None
    if occ_stream and sizing != "card":
        raise ValueError("occ_stream needs sizing='card' (the cardinality pass writes the stream)")
    if sizing == "card" and (heavy or occ_stream or not (capacity and bloom_words and list_capacity is not None)):
        sk = CardSketch(k, P, n_owners=n_owners, owner=owner, forward_only=forward_only, seed=seed, device=dev)
        if occ_stream:
            occ = OccStream(occ_capacity, device=dev) if occ_capacity is not None else \
                OccStream.for_windows(P, n_owners, 1, device=dev)
            while True:
                card = sk.run([packed], min_depth=min_depth, occ=occ)
                if not occ.overflowed():
                    break
                occ = OccStream(2 * max(occ.capacity, occ.entries()), device=dev)
        else:
            card = sk.run([packed], min_depth=min_depth)
        c_cap, c_bw, c_lcap = plan_sizes(card, n_hash=n_hash, device=dev, bloom_in_table=bloom_in_table)
        del sk
        if bypass or min_depth == 1:  # every distinct k-mer goes into the table
            c_cap = next_pow2(max(1024, int(card.distinct_hi() / 0.5)))
    elif sizing in ("card", "bound"):
        c_cap, c_lcap, c_bw = next_pow2(max(1024, 2 * P)), max(P, 1), next_pow2(max(64, P * 10 // 64))
    else:
        raise ValueError("sizing must be 'card' or 'bound'")
    cap = capacity or c_cap
    lcap = list_capacity if list_capacity is not None else c_lcap
    bw = bloom_words or c_bw
    for _ in range(retries + 1):
        kc = KmerCounter(k, cap, bw, lcap, n_hash=n_hash, min_depth=min_depth, ext_min=ext_min, n_owners=n_owners,
                         owner=owner, flags=flags, seed=seed, max_probe=max_probe, present_filter=present_filter,
                         heavy=card if heavy else None, bloom_in_table=bloom_in_table,
                         device=dev)
        out = Records(kc.capacity, device=dev)
        if occ is not None:
            kc.run_occ(occ, out, flags=export_flags, fused=fused)
        else:
            kc.run([packed], out, flags=export_flags, fused=fused)
        rc = kc.status()
        if rc == abi.HM_OK:
            res = out.to_numpy(sort=not (export_flags & abi.HM_EXPORT_SORTED))
            res["digest"] = out.digest_words()
            res["positions"] = P
            res["capacity"] = kc.capacity
            res["stats"] = kc.stats()
            res["n_heavy"] = kc.table.n_heavy
            if occ is not None:
                res["occ_entries"] = occ.entries()
                res["card_positions"] = card.positions
            return res
        if rc == abi.HM_ECAPACITY:
            st = int(kc.status_buf.item())
            if st & abi.HM_ST_TABLE_FULL:
                cap *= 2
            if st & abi.HM_ST_LIST_FULL:
                lcap *= 2
            continue
        abi.check(rc, "k-mer analysis")
    raise abi.HmError(abi.HM_ECAPACITY, "k-mer analysis", "still full after %d retries" % retries)
