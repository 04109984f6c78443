"""Batched k-mer analysis: many read sets in one persistent launch (C ABI
hm_batch_prepare / hm_batch_launch), replayed from a captured HIP graph.

Every set keeps its own packed reads, count table, Bloom filter,
first-occurrence list and export buffer (device tensors owned here).  The
same buffers also serve the plain per-set path (`run_plain`), so the two
forms can be compared set by set on identical memory.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import abi, kmer
from .kmer import KmerCounter, Records, next_pow2


# The first-occurrence list of every set keeps room for one partly used
# 256-entry chunk per wave of up to this many workgroups per CU, so any launch
# shape the autotuner tries (tune.LAUNCH_SPACE) fits the same buffers.
MAX_BLOCKS_PER_CU = 12


@dataclass
class Tuning:
    blocks_per_cu: int = 8
    tile_bases: int = 65536      # bases of reads per pass-1 item (staged in LDS 16384 at a time)
    list_per_item: int = 65536
    slots_per_item: int = 65536
    table_load: float = 0.45     # sizing: expected kept k-mers / capacity
    bloom_bits: float = 12.0     # sizing: Bloom bits per expected distinct k-mer
    n_hash: int = 4
    set_major: int = 2           # set by set, pass 2 lagging one set (cache-resident tables, few waits)
    bloom_in_table: bool = True  # sizing: the filter in the table's slots (32 bits each) or a separate one

    def struct(self) -> abi.BatchTuning:
        return abi.BatchTuning(self.blocks_per_cu, self.tile_bases, self.list_per_item, self.slots_per_item,
                               self.set_major)

    def key(self) -> tuple:
        return (self.blocks_per_cu, self.tile_bases, self.list_per_item, self.slots_per_item, self.table_load,
                self.bloom_bits, self.n_hash, self.set_major, self.bloom_in_table)


@dataclass
class SetSpec:
    """One read set: device-resident fixed-length reads and size estimates
    (expected distinct k-mers and k-mers seen at least twice)."""
    ascii: torch.Tensor
    qual: torch.Tensor
    read_len: int
    distinct_est: float
    kept_est: float

    @property
    def n_reads(self) -> int:
        return self.ascii.numel() // self.read_len


class _SetBuffers:
    def __init__(self, spec: SetSpec, k: int, params: dict, tuning: Tuning, device, plan: bool = True, qcut: int = 20,
                 qual_offset: int = 0):
        self.spec = spec
        n_bases = spec.n_reads * spec.read_len
        L = abi.lib()
        self.b2 = torch.empty(int(L.hm_bases2_words(n_bases)), dtype=torch.int64, device=device)
        self.nm = torch.empty(int(L.hm_mask_words(n_bases)), dtype=torch.int64, device=device)
        self.hq = torch.empty(int(L.hm_mask_words(n_bases)), dtype=torch.int64, device=device)
        bypass = params.get("min_depth", 2) == 1 or bool(params.get("flags", 0) & abi.HM_BLOOM_BYPASS)
        params = dict(params)
        in_table = bool(params.pop("bloom_in_table", tuning.bloom_in_table))  # an explicit choice wins
        if plan:  # sizes from a cardinality pass over the set's own reads
            kmer.pack_reads(spec.ascii, spec.qual, read_len=spec.read_len, qcut=qcut, qual_offset=qual_offset,
                            out=self.packed())
            sk = kmer.CardSketch(k, spec.n_reads * max(spec.read_len - k + 1, 0),
                                 n_owners=params.get("n_owners", 1), owner=params.get("owner", 0),
                                 forward_only=bool(params.get("flags", 0) & abi.HM_FORWARD_ONLY),
                                 seed=params.get("seed", kmer.DEFAULT_SEED), device=device)
            card = sk.run([self.packed()], min_depth=params.get("min_depth", 2))
            del sk
            distinct, kept = card.distinct_hi(), card.kept_hi()
            fp = kmer.bloom_fp_rate(tuning.bloom_bits, tuning.n_hash, word_bits=32 if in_table else 64)
            kept = kept + fp * max(distinct - kept, 0.0)
        else:  # the caller's size hints
            distinct, kept = spec.distinct_est, spec.kept_est
        keys = distinct if bypass else kept  # bypass keeps every distinct k-mer
        cap = next_pow2(max(1024, int(keys / tuning.table_load)))
        bw = next_pow2(max(64, int(distinct * tuning.bloom_bits / 64)))
        cus = torch.cuda.get_device_properties(device).multi_processor_count
        # + one partly used 256-entry chunk per wave of either form, for every launch shape
        lcap = int(distinct * (1.0 if plan else 1.2)) + cus * max(8, MAX_BLOCKS_PER_CU, tuning.blocks_per_cu) * 4 * 255
        self.kc = KmerCounter(k, cap, bw, lcap, n_hash=tuning.n_hash, bloom_in_table=in_table, device=device,
                              **params)
        self.out = Records(int(min(cap, keys * 1.3 + 1024)), device=device)

    def packed(self) -> kmer.Packed:
        return kmer.Packed(self.b2, self.nm, self.hq, None, self.spec.n_reads, self.spec.n_reads * self.spec.read_len,
                           self.spec.read_len)

    def struct(self) -> abi.BatchSet:
        kc = self.kc
        return abi.BatchSet(self.spec.ascii.data_ptr(), self.spec.qual.data_ptr(), self.spec.n_reads,
                            self.spec.read_len, self.b2.data_ptr(), self.nm.data_ptr(), self.hq.data_ptr(), kc.table,
                            kc.bloom, kc.list, self.out.struct())


class Batch:
    """A batch of read sets sharing one k-mer analysis parameter block."""

    def __init__(self, specs: list[SetSpec], k: int, qcut: int = 20, min_depth: int = 2, ext_min: int | None = None,
                 qual_offset: int = 0, export_flags: int = 0, tuning: Tuning | None = None, device="cuda",
                 plan: bool = True, **params):
        """plan: size every set's structures from a cardinality pass over its reads (else from the
        SetSpec size hints)."""
        self.device = torch.device(device)
        self.k, self.qcut, self.qual_offset, self.export_flags = k, qcut, qual_offset, export_flags
        self.tuning = tuning or Tuning()
        self.params = dict(min_depth=min_depth, ext_min=ext_min, **params)
        self.sets = [_SetBuffers(s, k, self.params, self.tuning, self.device, plan=plan, qcut=qcut,
                                 qual_offset=qual_offset) for s in specs]
        n = len(self.sets)
        wb = int(abi.lib().hm_batch_work_bytes(n))
        self.work = torch.empty(wb // 8 + 32, dtype=torch.int64, device=self.device)
        self.plan = abi.BatchPlan()
        self.graph = None
        self._prepare()

    def _prepare(self):
        arr = (abi.BatchSet * len(self.sets))(*[s.struct() for s in self.sets])
        self._arr = arr
        tu = self.tuning.struct()
        p = self.sets[0].kc.params
        work_ptr = (self.work.data_ptr() + 255) // 256 * 256
        abi.call("hm_batch_prepare", arr, len(self.sets), ctypes.byref(p), self.qual_offset, self.qcut,
                 self.export_flags, ctypes.byref(tu), work_ptr, self.work.numel() * 8 - (work_ptr - self.work.data_ptr()),
                 ctypes.byref(self.plan), kmer._stream())

    # ---- batched form
    def launch(self, stream=None):
        abi.call("hm_batch_launch", ctypes.byref(self.plan), kmer._stream(stream))

    def capture(self):
        """Capture one launch in a HIP graph (after a warm-up launch)."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.launch()
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    # ---- plain per-set form on the same buffers (the same kernels' work as five ABI calls per set:
    # pack, init, pass 1, pass 2, export with inline classification)
    def run_plain(self, stream=None):
        for sb in self.sets:
            kmer.pack_reads(sb.spec.ascii, sb.spec.qual, read_len=sb.spec.read_len, qcut=self.qcut,
                            qual_offset=self.qual_offset, stream=stream, out=sb.packed())
            sb.kc.run([sb.packed()], sb.out, flags=self.export_flags, stream=stream, fused=True)

    # ---- results
    def status(self) -> list[int]:
        torch.cuda.synchronize(self.device)
        return [sb.kc.status() for sb in self.sets]

    def digests(self) -> list[tuple]:
        torch.cuda.synchronize(self.device)
        return [(int(sb.out.n_out.item()),) + sb.out.digest_words() for sb in self.sets]

    def table(self, i: int) -> dict:
        return self.sets[i].out.to_numpy()

    def positions(self) -> int:
        return sum(sb.spec.n_reads * max(0, sb.spec.read_len - self.k + 1) for sb in self.sets)

    def device_bytes(self) -> int:
        return sum(sb.kc.bytes() + sb.b2.numel() * 8 * 2 for sb in self.sets)
