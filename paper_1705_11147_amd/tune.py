"""Autotuner of the batched form.

Chooses the launch shape of the persistent kernel (blocks per CU, pass-1
tile size, pass-2 and export item sizes) and the sizing of each set's
structures (table load factor, Bloom bits per distinct k-mer) by coordinate
descent: starting from the defaults, each parameter in turn is swept over its
candidates with the others fixed, and the fastest value is kept.  Every
candidate is timed with HIP events over `reps` launches on a sample of the
sets, and every candidate must give the same per-set digests (the output does
not depend on the tuning).  Results are cached in a JSON file keyed by
device, k, read length and set-size bucket.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import torch

from .batch import MAX_BLOCKS_PER_CU, Batch, SetSpec, Tuning

LAUNCH_SPACE = {
    "set_major": [2, 1, 3, 0],
    "blocks_per_cu": [4, 8, MAX_BLOCKS_PER_CU],  # the sets' list slack covers every value here
    "tile_bases": [16384, 32768, 65536, 131072],
    "list_per_item": [16384, 65536],
    "slots_per_item": [32768, 131072],
}
SIZING_SPACE = {
    "table_load": [0.3, 0.45, 0.6],
    "bloom_bits": [8.0, 12.0, 16.0],
    # with many more distinct than kept k-mers, the filter in the table (32 bits per 64-byte slot) makes
    # the table larger than its keys need, and the clear and the export sweep every slot
    "bloom_in_table": [True, False],
}


def _time(batch: Batch, reps: int) -> float:
    stream = torch.cuda.current_stream()
    batch.launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        batch.launch()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cache_key(specs: list[SetSpec], k: int) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    mean_bases = sum(s.ascii.numel() for s in specs) / max(1, len(specs))
    bucket = int(round(math.log2(max(mean_bases, 1))))
    return "%s|cu%d|k%d|L%d|n%d|2^%d" % (props.name, props.multi_processor_count, k, specs[0].read_len, len(specs),
                                          bucket)


def autotune(specs: list[SetSpec], k: int, sample: int = 16, reps: int = 2, cache_path: str | None = None,
             log=None, **batch_kw) -> tuple[Tuning, dict]:
    """Return (best tuning, report).  `specs` are the sets to tune for; a
    sample of them (spread over the size range) is what gets timed."""
    key = cache_key(specs, k)
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
            if key in cache:
                return Tuning(**cache[key]["tuning"]), {"cached": True, **cache[key]}
        except (OSError, ValueError, TypeError):
            pass
    order = sorted(range(len(specs)), key=lambda i: specs[i].ascii.numel())
    step = max(1, len(order) // sample)
    sub = [specs[i] for i in order[::step]][:sample]
    best = Tuning()
    trials = []
    rejected = []
    reference = None

    def run(tu: Tuning, batch: Batch | None = None):
        nonlocal reference
        b = batch or Batch(sub, k, tuning=tu, **batch_kw)
        if batch is not None:
            b.tuning = tu
            b._prepare()
        ms = _time(b, reps)
        st = b.status()
        if any(x != 0 for x in st):  # reported, never timed as a valid candidate
            rejected.append({"tuning": dataclasses.asdict(tu), "status": st})
            if log:
                log("tune %s: rejected, set statuses %s" % (tu.key(), sorted(set(st))))
            return None, b
        dig = b.digests()
        if reference is None:
            reference = dig
        elif dig != reference:
            raise AssertionError("autotuner: output changed with tuning %s" % (tu,))
        trials.append({"tuning": dataclasses.asdict(tu), "ms": ms})
        if log:
            log("tune %s: %.2f ms" % (tu.key(), ms))
        return ms, b

    best_ms, batch = run(best)
    for name, values in LAUNCH_SPACE.items():
        for v in values:
            if getattr(best, name) == v:
                continue
            tu = dataclasses.replace(best, **{name: v})
            ms, batch = run(tu, batch)
            if ms is not None and ms < best_ms:
                best, best_ms = tu, ms
        batch.tuning = best
    del batch
    torch.cuda.empty_cache()
    for name, values in SIZING_SPACE.items():
        for v in values:
            if getattr(best, name) == v:
                continue
            tu = dataclasses.replace(best, **{name: v})
            ms, b = run(tu)
            del b
            torch.cuda.empty_cache()
            if ms is not None and ms < best_ms:
                best, best_ms = tu, ms
    report = {"key": key, "tuning": dataclasses.asdict(best), "ms": best_ms, "sample_sets": len(sub),
              "trials": trials, "rejected": rejected}
    if cache_path:
        try:
            cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            cache = {}
        cache[key] = {"tuning": dataclasses.asdict(best), "ms": best_ms}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, report
