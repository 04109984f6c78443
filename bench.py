#!/usr/bin/env python3
"""Benchmark: k-mer analysis throughput (k-mers/s) on one MI355X.

One step = the whole path over one read set already resident in HBM (ASCII
bases + Phred bytes): pack -> cardinality pass (which also counts the
partition's first-level histogram) -> partition of the windows into LDS-sized
bins -> per bin, in workgroup memory: Bloom filter test + insert/count, the
deferred first occurrences, classify + export (the binned path).  The table
path's step (pack -> cardinality -> table/Bloom/list init -> pass 1 -> pass 2
-> classify + export) is timed beside it as a sub-record, and both must give
the same export.  The headline workload is the mid-size read set: 100 Mbp synthetic
genome with 5% segmental repeats, 20M reads of 150 bp (30x), 0.5% end-biased
substitution errors, Phred ~ clamp(N(32,6),2,41), k=51, Q20, min depth 2.

Prints ONE JSON line: the throughput; the dominant kernel's place on the HBM
roofline; one key shard of the timed export checked against the CPU oracle;
the oracle timed on a bounded sample (whose table the GPU must reproduce);
and, as sub-records, the tiny read set (checked against the oracle in full, the oracle timed on
one host thread and on all of them), the batched form (64 read sets) against the plain form,
the serving loop, and one GPU's share of the human-scale run (owner 0 of 16,
ten 64M-read batches; the binned path from the owned-occurrence stream, the
table path beside it) with a sub-shard of its table checked against the
oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-mers/sec k-mer analysis (bit-exact); batched vs plain; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
LINE = 64  # bytes moved by one random access (HBM/L2 line granularity)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads() -> int:
    return len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


RECORD_FIELDS = ("key_hi", "key_lo", "count", "tl", "tr", "cls_l", "cls_r")


def device_rows(rec, idx) -> dict:
    """Host copies of the records `idx` (a device index tensor) of an export buffer, in key order."""
    n = int(idx.numel())
    t = {"key_hi": rec.key_hi[idx].cpu().numpy().view(np.uint64),
         "key_lo": rec.key_lo[idx].cpu().numpy().view(np.uint64),
         "count": rec.count[idx].cpu().numpy().view(np.uint32),
         "tl": rec.tl.view(-1, 4)[idx].cpu().numpy().view(np.uint32).reshape(n, 4),
         "tr": rec.tr.view(-1, 4)[idx].cpu().numpy().view(np.uint32).reshape(n, 4),
         "cls_l": rec.cls_l[idx].cpu().numpy(), "cls_r": rec.cls_r[idx].cpu().numpy()}
    order = np.lexsort((t["key_lo"], t["key_hi"]))
    return {x: v[order] for x, v in t.items()}


def same_records(a: dict, b: dict) -> bool:
    """Field-by-field equality of two key-ordered record sets."""
    return len(a["count"]) == len(b["count"]) and all(np.array_equal(a[f], b[f]) for f in RECORD_FIELDS)


def source_digest(paths) -> str:
    """sha256 over the concatenated source files that define a kernel."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


PASS1_SOURCES = [os.path.join(ROOT, "paper_1705_11147_amd", "csrc", f) for f in ("hm_device.h", "hm_kmer.hip")]


def profiled_traffic(profile: str, sources=PASS1_SOURCES):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    summary, or None when the kernel source changed since it was measured."""
    try:
        text = open(profile).read()
        digest = source_digest(sources)
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_bytes", "source_sha")))
    if fields.get("source_sha256", "").strip() != digest or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"].strip())


def measure_sorted_export(kc, out, k, n_records, ref_digest, stream, log, reps=3):
    """Time the export with and without HM_EXPORT_SORTED on the bench table (outside the timed
    step: the path's output is an unordered record set) and check the device's order."""
    import torch
    from paper_1705_11147_amd import abi
    flags = abi.HM_EXPORT_CLASSIFY
    kc.export(out, flags | abi.HM_EXPORT_SORTED)  # allocates the scratch once
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        kc.export(out, flags)
        ev[2 * i + 1].record(stream)
        kc.export(out, flags | abi.HM_EXPORT_SORTED)
        ev[2 * i + 2].record(stream)
    torch.cuda.synchronize()
    abi.check(kc.status(), "sorted export")
    plain = float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]))
    srt = float(np.mean([ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(reps)]))
    n = int(out.n_out.item())
    assert n == n_records and out.digest_words() == ref_digest, "sorted export changed the record set"
    hi, lo = out.key_hi[:n], out.key_lo[:n] ^ (-2 ** 63)  # flip the sign bit: signed order = unsigned order
    ordered = bool(((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))).all().item())
    assert ordered, "sorted export is not in key order"
    kw = 2 if 2 * k > 64 else 1
    rec = 8 * kw + 4  # key words + 4-byte index
    # algorithmic bytes per record on top of the plain export: the export writes a 48-byte staging
    # line instead of 38 record bytes (+10); a counting pass reads the digit's key word for the tile
    # counts, then reads and writes the keys and index; the gather reads the index and one 64-byte
    # line and writes 38 record bytes, and moves the keys when they end in the scratch
    if 2 * k >= 32:  # two grouping passes, the group starts (one key word), each group read and written once
        passes = 2
        per_rec = 10 + passes * (8 + 2 * rec) + 8 + 2 * rec + (4 + 64 + 38 + 2 * 8 * kw)
    else:
        passes = (2 * k + 7) // 8
        copy = (passes & 1) * 8 * kw
        per_rec = 10 + passes * (8 + 2 * rec) + (4 + 64 + 38 + 2 * copy)
    sort_ms = srt - plain
    res = {"records": n, "key_bits": 2 * k, "counting_passes": passes, "export_ms": round(plain, 3),
           "export_sorted_ms": round(srt, 3), "sort_ms": round(sort_ms, 3),
           "sort_records_per_s": round(n / (sort_ms / 1000), 1), "bytes_per_record": per_rec,
           "sort_algorithmic_GBps": round(n * per_rec / (sort_ms / 1000) / 1e9, 1), "order_checked": ordered}
    log("sorted export: %s" % res)
    return res


def run_batched(args, dev, log):
    """64 read sets (0.5-8 Mbp genomes, 10-60x, 150 bp, 1% errors, k=31): the
    batched persistent form replayed from a HIP graph against the plain
    per-set path on the same buffers; outputs compared set by set."""
    import torch
    from paper_1705_11147_amd import abi, synth, tune
    from paper_1705_11147_amd.batch import Batch, SetSpec

    t0 = time.time()
    ws = synth.batched_sets(n_sets=args.batch_sets, scale=args.batch_scale)
    specs = []
    for w in ws:
        r = w.reads()
        d, kept = w.size_estimates()
        specs.append(SetSpec(torch.from_numpy(r.ascii).to(dev), torch.from_numpy(r.qual).to(dev), r.read_len, d,
                             kept))
        del r
    k = ws[0].params.k
    log("batched: %d sets generated in %.1fs" % (len(ws), time.time() - t0))
    t1 = time.time()
    # tuned on the whole batch (a sample of sets timed with few launches chose differently from run to run)
    best, report = tune.autotune(specs, k, sample=len(specs), reps=3, log=log)
    tune_s = time.time() - t1
    log("batched: tuned in %.1fs -> %s" % (tune_s, best.key()))
    torch.cuda.empty_cache()
    b = Batch(specs, k, tuning=best, device=dev)
    b.launch()
    st = b.status()
    if any(x != abi.HM_OK for x in st):
        raise RuntimeError("batched run failed: statuses %s" % st)
    ref = b.digests()
    b.capture()
    positions = b.positions()
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_b = timed(b.replay, args.steps)
    assert b.digests() == ref, "batched output changed between replays"
    ms_p = timed(b.run_plain, args.steps)
    st = b.status()
    same = st == [abi.HM_OK] * len(st) and b.digests() == ref
    assert same, "batched and plain forms disagree (statuses %s)" % sorted(set(st))
    return {"workload": "batched-64-sets-0.5to8Mbp-10to60x-150bp-k31", "sets": len(ws), "positions": positions,
            "batched_kmers_per_s": round(positions / (ms_b / 1000), 1), "batched_ms": round(ms_b, 3),
            "plain_kmers_per_s": round(positions / (ms_p / 1000), 1), "plain_ms": round(ms_p, 3),
            "speedup": round(ms_p / ms_b, 3), "outputs_identical": bool(same),
            "tuning": dict(zip(["blocks_per_cu", "tile_bases", "list_per_item", "slots_per_item", "table_load",
                                "bloom_bits", "n_hash", "set_major", "bloom_in_table"], best.key())),
            "tune_s": round(tune_s, 1), "tune_trials": len(report.get("trials", [])),
            "tune_ms": {"best": round(report["ms"], 3),
                        "bloom_in_table_false": min([t["ms"] for t in report.get("trials", [])
                                                     if not t["tuning"]["bloom_in_table"]] or [None])},
            "form": "hipGraph replay of clear + pack + persistent counting kernel + export, vs 64 x 5 plain calls"}


def run_heavy(args, dev, log):
    """Heavy hitters (the mid workload with 2% of the genome in tandem satellite arrays, so that a
    few k-mers hold millions of windows each): pass 1 with the cardinality pass's heavy list counted
    in workgroup-local memory, against the same pass with every occurrence going through the table;
    both tables must be identical."""
    import torch
    from paper_1705_11147_amd import abi, kmer, synth

    t0 = time.time()
    w = synth.mid_heavy()
    r = w.reads()
    p = w.params
    L, k = r.read_len, p.k
    positions = r.n_reads * (L - k + 1)
    ascii = torch.from_numpy(r.ascii).to(dev)
    qual = torch.from_numpy(r.qual).to(dev)
    del r
    packed = kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut)
    del ascii, qual
    card = kmer.CardSketch(k, positions, device=dev).run([packed], min_depth=p.min_depth)
    abi.check(card.status, "cardinality pass (heavy workload)")
    cap, bw, lcap = kmer.plan_sizes(card, device=dev)
    log("heavy: %s generated and sized in %.1fs, %d heavy hitters" % (w.name, time.time() - t0, card.n_heavy))
    out = {"workload": w.name, "positions": positions, "heavy_hitters": card.n_heavy}
    digests = {}
    for name, heavy in (("heavy_in_lds", card), ("through_table", None)):
        kc = kmer.KmerCounter(k, cap, bw, lcap, min_depth=p.min_depth, heavy=heavy, device=dev)
        rec = kmer.Records(int(cap * 0.6), device=dev)
        ms = []
        for i in range(1 + args.steps):  # one untimed
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            kc.reset()
            ev[0].record()
            kc.insert(packed)
            ev[1].record()
            kc.count()
            kc.export(rec, abi.HM_EXPORT_CLASSIFY)
            ev[2].record()
            torch.cuda.synchronize()
            if i:
                ms.append((ev[0].elapsed_time(ev[1]), ev[0].elapsed_time(ev[2])))
        abi.check(kc.status(), "heavy workload (%s)" % name)
        st = kc.stats()
        digests[name] = (rec.digest_words(), int(rec.n_out.item()))
        out[name] = {"pass1_ms": round(float(np.mean([x[0] for x in ms])), 3),
                     "pass1_to_export_ms": round(float(np.mean([x[1] for x in ms])), 3),
                     "wide_counts_per_position": round(st["wide_counts"] / positions, 5),
                     "heavy_local_per_position": round(st["heavy_local"] / positions, 5)}
        del kc, rec
        torch.cuda.empty_cache()
    same = digests["heavy_in_lds"] == digests["through_table"]
    assert same, "the heavy-hitter treatment changed the table"
    out["outputs_identical"] = bool(same)
    out["pass1_gain"] = round(out["through_table"]["pass1_ms"] / out["heavy_in_lds"]["pass1_ms"], 3)
    log("heavy: pass 1 %.1f ms with the heavy list in LDS, %.1f ms through the table" % (
        out["heavy_in_lds"]["pass1_ms"], out["through_table"]["pass1_ms"]))
    return out


def run_tiny(args, dev, log, steps=50):
    """The tiny read set (1 Mbp genome, 200k reads of 100 bp, k=21): the whole step on the GPU,
    its table against the oracle's in full, and the oracle timed on one host thread and on all of
    them.  The step is bound by kernel latency, not by HBM, so no roofline fraction is claimed."""
    import torch
    import oracle
    from paper_1705_11147_amd import abi, kmer, synth

    w = synth.tiny()
    r = w.reads()
    p = w.params
    L, k = r.read_len, p.k
    positions = r.n_reads * (L - k + 1)
    stream = torch.cuda.current_stream()
    ascii = torch.from_numpy(r.ascii).to(dev)
    qual = torch.from_numpy(r.qual).to(dev)
    packed = kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut)
    sketch = kmer.CardSketch(k, positions, device=dev)
    card = sketch.run([packed], min_depth=p.min_depth)
    abi.check(card.status, "cardinality pass (tiny)")
    cap, bw, lcap = kmer.plan_sizes(card, device=dev)
    kc = kmer.KmerCounter(k, cap, bw, lcap, min_depth=p.min_depth, heavy=card, device=dev)
    out = kmer.Records(int(cap * 0.6), device=dev)

    stages = ["pack", "card", "init", "pass1", "pass2", "classify_export"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut, out=packed)
        mark(1)
        sketch.reset()
        sketch.update(packed)
        sketch.summarize(min_depth=p.min_depth)
        mark(2)
        kc.reset()
        mark(3)
        kc.insert(packed)
        mark(4)
        kc.count()
        mark(5)
        kc.export(out, abi.HM_EXPORT_CLASSIFY)
        mark(6)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    # whole steps back to back, then the same steps with an event between stages
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    sev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(10)]
    for e in sev:
        step(e)
    torch.cuda.synchronize()
    abi.check(kc.status(), "k-mer analysis (tiny)")
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    stage_ms = {x: round(float(np.median([e[i].elapsed_time(e[i + 1]) for e in sev])), 4)
                for i, x in enumerate(stages)}
    got = out.to_numpy()
    threads = host_threads()
    runs = {}
    for name, th, sort_count in (("sort_counted_1_thread", 1, True), ("sort_counted_all_threads", threads, True),
                                 ("hash_map_1_thread", 1, False)):
        res = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=p.qcut, min_depth=p.min_depth, n_threads=th,
                         sort_count=sort_count)
        assert same_records(got, res) and res["positions"] == positions, \
            "the tiny workload's GPU table disagrees with the oracle (%s)" % name
        runs[name] = {"threads": th, "s": round(res["seconds"], 3),
                      "kmers_per_s": round(positions / res["seconds"], 1)}
    med = float(np.median(step_ms))
    res = {"workload": w.name, "positions": positions, "kept_kmers": len(got["count"]), "table_slots": kc.capacity,
           "steps": steps, "ms_per_step": {"median": round(med, 4), "p10": round(float(np.percentile(step_ms, 10)), 4),
                                           "p90": round(float(np.percentile(step_ms, 90)), 4)},
           "kmers_per_s": round(positions / (med / 1000), 1), "stage_ms": stage_ms,
           "bound": "kernel latency (the tables fit in cache); no roofline fraction claimed",
           "oracle_identical": True, "oracle": runs, "host_cpu": cpu_model()}
    log("tiny: %.3f ms/step (%.3g k-mers/s), stages %s; oracle %s" % (med, positions / (med / 1000), stage_ms, runs))
    del kc, out, packed, ascii, qual
    return res


RECORD_OUT_BYTES = 54  # an exported record: key 16 + count 4 + two tally arrays 32 + two class bytes
BIN_SOURCES = [os.path.join(ROOT, "paper_1705_11147_amd", "csrc", f) for f in ("hm_device.h", "hm_bins.h", "hm_roll.h", "hm_bins.hip")]


def run_binned_step(args, dev, log, ascii, qual, packed, sketch, card, positions, L, p, stream, ref_digest,
                    n_records, method_bpp):
    """The binned path as the step: pack, cardinality pass, partition into LDS-sized bins
    (hm_bin_kmers), per-bin Bloom filter + table + classification + export in workgroup memory
    (hm_count_bins), and, when a bin did not fit, its records through the table path (checked
    every step: the spill count is read back).  Returns the figures and the export buffer."""
    import torch
    from paper_1705_11147_amd import abi, kmer

    g, b = kmer.plan_bins(card.distinct_hi(), card.kept_hi(), p.min_depth == 1)
    bc = kmer.BinnedCounter(p.k, positions, g, b, min_depth=p.min_depth, device=dev)
    out = kmer.Records(int(n_records * 1.2) + 4096, device=dev)
    stages = ["pack", "card", "partition", "count"]
    spilled = [0]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut, out=packed)
        mark(1)
        sketch.reset()
        sketch.update(packed, bins=bc)  # also counts the partition's first-level histogram
        sketch.summarize(min_depth=p.min_depth)
        mark(2)
        bc.bin(packed, counted=True)
        mark(3)
        bc.count(out)
        mark(4)
        n_sp = bc.spilled()  # synchronizes; a spilled bin is counted by the table path
        if n_sp:
            spilled[0] += n_sp
            bc.finish(out)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(args.steps)]
    spilled[0] = 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    abi.check(bc.status(), "binned k-mer analysis (timed steps)")
    same = out.digest_words() == ref_digest and int(out.n_out.item()) == n_records
    assert same, "the binned export differs from the table path's"
    stage_ms = {x: float(np.mean([events[s][i].elapsed_time(events[s][i + 1]) for s in range(args.steps)]))
                for i, x in enumerate(stages)}
    step_ms = np.array([events[s][0].elapsed_time(events[s][len(stages)]) for s in range(args.steps)])
    st = bc.stats()
    # the longest kernel: k_count_bins (one launch of hm_count_bins, timed by the events around it).
    # Algorithmic bytes: every record read once, every kept record written
    cnt_ms = stage_ms["count"]
    alg = RECORD_OUT_BYTES * n_records + 16 * positions
    achieved = alg / (cnt_ms / 1000) / 1e9
    med = float(np.median(step_ms))
    roofline = {"kernel": "k_count_bins (per-bin Bloom filter, table, classification and export in LDS)",
                "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(os.path.join(ROOT, "profiles", "k_count_bins_mid_k51_traffic.md"),
                                            BIN_SOURCES) if args.scale == 1.0 and args.workload == "mid" else None,
                "bytes_per_position": round(alg / positions, 2),
                "model": "16 B read per record + %d B written per kept k-mer" % RECORD_OUT_BYTES,
                "kernel_ms": round(cnt_ms, 3),
                "frac_step_method_model": round(method_bpp * positions / (med / 1000) / 1e9 / HBM_PEAK_GBS, 4),
                "method_model": "(1 + s) * 2g + g bytes per position (g = 64 B) over the whole step: the random "
                                "line accesses the table design makes, which the binned design replaces"}
    res = {"value": round(positions * args.steps / elapsed, 1), "ms_per_step": round(elapsed * 1000 / args.steps, 3),
           "stage_ms": {x: round(v, 3) for x, v in stage_ms.items()},
           "step_ms": {"median": round(med, 3), "p10": round(float(np.percentile(step_ms, 10)), 3),
                       "p90": round(float(np.percentile(step_ms, 90)), 3), "n": int(args.steps)},
           "bins": {"group_bits": g, "bin_bits": b, "n_bins": 1 << (g + b), "records_padded": bc.capacity,
                    "spilled_records_per_step": spilled[0] // max(args.steps, 1), **st},
           "roofline": roofline, "same_as_table_path": bool(same)}
    log("binned step: %.2f ms (%s), count kernel %.2f ms" % (med, ", ".join("%s %.2f" % kv for kv in stage_ms.items()),
                                                           cnt_ms))
    return res, bc, out


def run_serving(args, dev, log):
    """Poisson arrivals (20 jobs/s) of hexaploid-like k-mer analysis jobs
    (ancestor log-U[1,50] Mbp + 3 homeologs at 1.5%, 30x of 150 bp, 0.5%
    errors, k=51), payloads in pinned host memory, served with continuous
    batching; the same job stream one job at a time (FIFO) for comparison."""
    import torch
    from paper_1705_11147_amd import synth
    from paper_1705_11147_amd.serve import GpuBackend, Scheduler, make_jobs, summarize

    t0 = time.time()
    _, builders = synth.serving_jobs(n_jobs=args.serve_pool, rate=args.serve_rate, scale=args.serve_scale)
    pool = [b() for b in builders]
    jobs, positions = make_jobs(pool, n_jobs=args.serve_jobs, rate=args.serve_rate)
    del pool
    log("serving: %d pooled jobs, %d arrivals prepared in %.1fs" % (args.serve_pool, len(jobs), time.time() - t0))
    budget = int(args.serve_budget_gb * 2 ** 30)
    out = {"workload": "serving-hexaploid-1to50Mbp-x3-30x-150bp-k51-poisson%gps" % args.serve_rate,
           "scale": args.serve_scale, "pool_jobs": args.serve_pool, "budget_GiB": args.serve_budget_gb}
    # the backend reserves the whole budget once (its arena), outside the timed runs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    be = GpuBackend(51, device=dev, memory_bytes=budget)
    # warm-up: one small job through the backend (stream, kernels)
    Scheduler(be, budget, 1).run([min(jobs, key=lambda j: j.n_bases)])
    for name, slots in (("continuous", args.serve_slots), ("fifo_one_at_a_time", 1)):
        torch.cuda.synchronize()
        be.arena.peak = be.arena.used
        spills = be.arena.spills
        # continuous: the next jobs plan while others count; one at a time: nothing overlaps a job
        sch = Scheduler(be, budget, slots,
                        max_planning=args.serve_planners if slots > 1 else 1, plan_while_busy=slots > 1)
        m0 = torch.cuda.memory_stats(dev)
        recs = sch.run(jobs)
        m1 = torch.cuda.memory_stats(dev)
        bad = [r.job for r in recs if r.status != 0 or r.result is None]
        assert not bad, "serving (%s): jobs %s failed" % (name, bad[:10])
        res = summarize(recs, positions, sch.trace)
        res["slots"] = slots
        res["planners"] = args.serve_planners if slots > 1 else 1
        # caching allocator during the run: device allocations, and retries (a retry frees the
        # cached blocks and synchronizes the device)
        for key, name_ in (("num_device_alloc", "device_allocs"), ("num_alloc_retries", "alloc_retries"),
                           ("num_sync_all_streams", "allocator_syncs")):
            if key in m1:
                res[name_] = int(m1[key] - m0.get(key, 0))
        res["arena_peak_GiB"] = be.arena.peak / 2 ** 30
        res["arena_spills"] = be.arena.spills - spills
        out[name] = {x: (round(v, 3) if isinstance(v, float) else v) for x, v in res.items()}
        log("serving %s: p50 %.1f ms p99 %.1f ms, %.3g k-mers/s" % (name, res["p50_ms"], res["p99_ms"],
                                                                     res["kmers_per_s"]))
        if name == "continuous":
            results = {r.job: r.result for r in recs}
        else:
            same = all(results[r.job] == r.result for r in recs)
            assert same, "a job's output differs between the continuous mix and one-at-a-time serving"
            out["identical_alone_vs_mix"] = bool(same)
    return out


def measure_contigs(kc, k, n_records, stream, log, reps=3, rates=None):
    """Time contig generation (hm_contigs) over the UU records of the bench table, outside the timed
    step, and check that the contigs hold every UU k-mer once.  With the measured random-access
    rates (`rates`: ops/s of loads and atomics, copy bytes/s), price the call's accesses at them:
    the random-access ceiling of this call, and the fraction of it reached."""
    import torch
    from paper_1705_11147_amd import abi, kmer
    uu = kmer.Records(n_records, device=kc.device)
    kc.export(uu, abi.HM_EXPORT_CLASSIFY | abi.HM_EXPORT_UU_ONLY, digest=False)
    abi.check(kc.status(), "UU export")
    n_uu = int(uu.n_out.item())
    cs = kmer.ContigSet(uu.capacity, k, device=kc.device)
    st = cs.run(uu)  # sizes the outputs
    assert st == 0, "contig generation status 0x%x" % st
    ref = tuple(int(x) for x in cs.counts.cpu().numpy())
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        cs.launch(uu, stream=stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
    assert int(cs.status_buf.item()) == 0 and tuple(int(x) for x in cs.counts.cpu().numpy()) == ref
    nc, nb = ref
    assert nb - nc * (k - 1) == n_uu, "contigs do not hold every UU k-mer once"
    lens = (cs.off[1:nc + 1] - cs.off[:nc]).sort(descending=True).values
    csum = lens.cumsum(0)
    n50 = int(lens[int((csum >= (nb + 1) // 2).nonzero()[0].item())].item()) if nc else 0
    t = float(np.median(ms))
    res = {"uu_kmers": n_uu, "contigs": nc, "bases": nb, "n50": n50, "longest": int(lens[0].item()) if nc else 0,
           "ms": round(t, 3), "uu_kmers_per_s": round(n_uu / (t / 1000), 1),
           "work_bytes": int(cs.work.numel() * 8)}
    # accesses per call (line granular, first probes only), per UU k-mer u and per reading h = 2u:
    #   index: a probe load and a claiming CAS per u;  link: two neighbour slot loads per u;
    #   walk 1 (lengths) and walk 2 (copy into runs): a successor load per h each;
    #   rulers (1 in 32 k-mers and the chain heads): a few words each, not counted;
    # plus the streamed bytes: the index fill (64 bytes per record of the buffer's capacity) and
    # per u about 90 bytes: keys and classes read twice, links written, runs written and read, the
    # contig bases
    cap = uu.capacity
    loads, stores, atomics = 7 * n_uu, 0, n_uu
    seq_bytes = 64 * cap + 90 * n_uu + nb
    res["random_ops_per_uu_kmer"] = round((loads + stores + atomics) / max(n_uu, 1), 2)
    res["achieved_random_Gops"] = round((loads + stores + atomics) / (t / 1000) / 1e9, 2)
    if rates:
        model_s = (loads + stores) / rates["load"] + atomics / rates["atomic_add"] + seq_bytes / rates["copy_Bps"]
        res["roofline"] = {"bound": "random access (measured rates)", "ceiling_ms": round(model_s * 1000, 2),
                           "frac_of_measured_ceiling": round(model_s * 1000 / t, 4),
                           "load_Gops": round(rates["load"] / 1e9, 2),
                           "atomic_Gops": round(rates["atomic_add"] / 1e9, 2),
                           "seq_bytes_per_uu_kmer": round(seq_bytes / max(n_uu, 1), 1)}
    log("contig generation: %s" % res)
    del cs, uu
    return res


def owner_zero_mask(key_hi, key_lo, bits: int):
    """Records of owner 0 of 2^bits under the owner map of hm_params_t (own = the top bits of
    H = (key_lo ^ key_hi * 0x9E3779B97F4A7C15) * 0xD1B54A32D192ED03 mod 2^64), computed with
    torch on the device: wrapping int64 products are the unsigned 64-bit ones, and the shift is
    made logical by masking.  A checker for the sub-shard comparison, outside the library."""
    import torch

    def s64(c):
        return c - (1 << 64) if c >= 1 << 63 else c

    def srl(x, n):
        return (x >> n) & ((1 << (64 - n)) - 1)

    h = (key_lo ^ key_hi * s64(0x9E3779B97F4A7C15)) * s64(0xD1B54A32D192ED03)
    return srl(h, 64 - bits) == 0 if bits > 0 else torch.ones_like(h, dtype=torch.bool)


def run_human_share(args, dev) -> dict:
    """One GPU's share of the human-scale run at its real shape (owner 0 of 16; reads in
    64M-read batches kept packed on the device), timed from the cardinality pass to the exported
    table.  The cardinality pass writes the owned occurrences to a stream that pass 1 reads.
    Checked against the CPU oracle on the 1/64 sub-shard owner 0 of 1024 (the owners nest): the
    oracle counts every batch's windows as the batch is generated (oracle.Accumulator, the
    sort-counted scheme on every host core), and the sub-shard's records of the GPU table must
    equal its records field by field."""
    import torch
    import oracle
    from paper_1705_11147_amd import abi, kmer, synth

    t0 = time.time()
    w = synth.human_share(scale=args.human_scale)
    p = w.params
    L, k = w.read_len, p.k
    nb = w.meta["batch_reads"]
    cuts = list(range(0, w.n_reads, nb)) + [w.n_reads]
    log("workload %s: genome %.3g bp, %d reads in %d batches (genome built in %.1fs)" % (
        w.name, w.meta["G"], w.n_reads, len(cuts) - 1, time.time() - t0))
    sub_bits = 10  # the checked sub-shard: owner 0 of 2^10, inside owner 0 of 16
    threads = host_threads()
    # every key of the sub-shard (keep_all), so that the counts also give its exact occurrence total
    acc = None if args.no_human_oracle else oracle.Accumulator(
        k, qcut=p.qcut, min_depth=p.min_depth, n_owners=1 << sub_bits, owner=0, sort_count=True, n_threads=threads,
        keep_all=True)
    packs, gen_s, up_ms, pack_ms = [], 0.0, 0.0, 0.0
    for b in range(len(cuts) - 1):
        t1 = time.time()
        r = w.reads(r0=cuts[b], n=cuts[b + 1] - cuts[b])
        gen_s += time.time() - t1
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        ascii = torch.from_numpy(r.ascii).to(dev)
        qual = torch.from_numpy(r.qual).to(dev)
        e[1].record()
        packs.append(kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut))
        e[2].record()
        if acc is not None:  # the oracle counts this batch on the host while the device packs it
            acc.add(r.ascii, r.qual, r.offsets())
        torch.cuda.synchronize()
        up_ms += e[0].elapsed_time(e[1])
        pack_ms += e[1].elapsed_time(e[2])
        del ascii, qual, r
        log("batch %d of %d: %d reads generated, uploaded and packed%s" % (
            b + 1, len(cuts) - 1, cuts[b + 1] - cuts[b], "; oracle %.1fs so far" % acc.seconds if acc else ""))
    torch.cuda.empty_cache()
    scanned = w.n_reads * (L - k + 1)
    sketch = kmer.CardSketch(k, scanned, n_owners=p.n_owners, owner=p.owner, device=dev)
    use_occ = not args.no_occ_stream
    occ = kmer.OccStream.for_windows(scanned, p.n_owners, len(packs), device=dev) if use_occ else None
    card = sketch.run(packs, min_depth=p.min_depth, occ=occ)
    abi.check(card.status, "cardinality pass")
    if occ is not None and occ.overflowed():  # the share was larger than planned: rerun with room for it
        occ = kmer.OccStream(card.positions + kmer.OccStream.slack(len(packs), dev), device=dev)
        card = sketch.run(packs, min_depth=p.min_depth, occ=occ)
    cap, bloom_words, list_cap = kmer.plan_sizes(card, pass1_launches=1 if use_occ else len(packs), device=dev)
    kc = kmer.KmerCounter(k, cap, bloom_words, list_cap, n_owners=p.n_owners, owner=p.owner, heavy=card, device=dev)
    out = kmer.Records(int(min(kc.capacity, card.kept_hi() * 1.3 + 1024)), device=dev)
    log("owned: %.4g windows, %.4g distinct (HLL) -> table 2^%d slots (%.1f GB), list %.3g entries%s" % (
        card.positions, card.estimate, kc.capacity.bit_length() - 1, kc.capacity * 64 / 1e9, list_cap,
        ", stream %.3g entries (%.1f GB)" % (occ.capacity, occ.capacity * 17 / 1e9) if occ else ""))
    stages = ["card", "init", "pass1", "pass2", "classify_export"]

    def step(ev):
        ev[0].record()
        sketch.reset()
        if occ is not None:
            occ.reset()
        for pk in packs:
            sketch.update(pk, occ=occ)
        sketch.summarize(min_depth=p.min_depth)
        ev[1].record()
        kc.reset()
        ev[2].record()
        if occ is not None:  # pass 1 reads the owned occurrences the cardinality pass wrote
            kc.insert_occ(occ)
        else:
            for pk in packs:
                kc.insert(pk)
        ev[3].record()
        kc.count()
        ev[4].record()
        kc.export(out, abi.HM_EXPORT_CLASSIFY)
        ev[5].record()

    n_steps = max(1, min(args.steps, 3))
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(n_steps + 1)]
    digests = []
    for s in range(n_steps + 1):  # the first is a warm-up
        step(events[s])
        torch.cuda.synchronize()
        abi.check(kc.status(), "human share step")
        digests.append(out.digest_words())
        log("step %d of %d done" % (s + 1, n_steps + 1))
    assert len(set(digests)) == 1, "the human-share table changed between steps"
    timed = events[1:]
    stage_ms = {x: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in timed])) for i, x in enumerate(stages)}
    step_ms = float(np.mean([ev[0].elapsed_time(ev[len(stages)]) for ev in timed]))
    n_rec = int(out.n_out.item())
    st = kc.stats()
    owned = st["occurrences"]

    check, cpu = None, None
    if acc is not None:
        t2 = time.perf_counter()
        every = acc.finish()
        sub_owned = int(every["count"].sum(dtype=np.uint64))  # owned occurrences of the sub-shard
        kept = every["count"] >= p.min_depth
        exp = {f: every[f][kept] for f in RECORD_FIELDS}
        exp["positions"] = every["positions"]
        del every
        sel = owner_zero_mask(out.key_hi[:n_rec], out.key_lo[:n_rec], sub_bits).nonzero().squeeze(1)
        got = device_rows(out, sel)
        same = same_records(got, exp)
        log("sub-shard owner 0 of %d: %d records in the GPU table, %d from the oracle, identical: %s (oracle %.1fs)" % (
            1 << sub_bits, len(got["count"]), len(exp["count"]), same, acc.seconds))
        assert same, "the human-share table disagrees with the oracle on its sub-shard"
        assert exp["positions"] == scanned
        check = {"sub_shard": "owner 0 of %d (1/%d of the share's keys)" % (1 << sub_bits, (1 << sub_bits) // 16),
                 "records": len(got["count"]), "oracle_identical": same, "compare_s": round(time.perf_counter() - t2, 1)}
        cpu = {"value": round(sub_owned / acc.seconds, 1), "unit": "k-mers/s", "cores": threads, "kind": "oracle",
               "sample": "the sub-shard owner 0 of %d: all %.3g windows of the ten batches scanned, its %d owned "
                         "occurrences counted (sort-counted, %d threads, %.1fs); %s" % (
                             1 << sub_bits, scanned, sub_owned, threads, acc.seconds, cpu_model()),
               "scanned_windows_per_s": round(scanned / acc.seconds, 1)}
    table_slots = kc.capacity
    binned = None
    if occ is not None and not args.no_binned_share and k <= 61:
        del kc, out  # the binned structures take the table's place in HBM
        torch.cuda.empty_cache()
        try:
            binned = run_binned_share(args, dev, packs, sketch, occ, card, p, k, digests[0], n_rec, owned)
        except torch.cuda.OutOfMemoryError as e:  # reported, not fatal: the table path's figures stand
            binned = {"error": "out of device memory: %s" % str(e).splitlines()[0]}
        torch.cuda.empty_cache()
    g = LINE
    s_seen = 1.0 - st["deferred"] / max(owned, 1)
    bpp = (1.0 + s_seen) * 2 * g + g
    rec = {
        "metric": "owned k-mers/s k-mer analysis, one GPU's share of the human-scale run (bit-exact)",
        "value": round(owned / (step_ms / 1000), 1), "unit": "k-mers/s", "steps": n_steps, "warmup": 1,
        "ms_per_step": round(step_ms, 3),
        "config": {"workload": w.name, "genome_bp": int(w.meta["G"]), "reads": w.n_reads, "read_len": L, "k": k,
                   "n_owners": p.n_owners, "owner": p.owner, "batches": len(packs),
                   "scanned_positions": scanned, "owned_positions": owned,
                   "scanned_positions_per_s": round(scanned / (step_ms / 1000), 1),
                   "kept_kmers": n_rec, "table_slots": table_slots, "list_capacity": list_cap,
                   "occ_stream_entries": occ.capacity if occ else 0, "hll_estimate": round(card.estimate, 1),
                   "step": "cardinality pass writing the owned occurrences + init + pass 1 over them + pass 2 + "
                           "classify/export; packed reads resident in HBM" if occ else
                           "cardinality + init + pass 1 over every batch + pass 2 + classify/export; packed reads "
                           "resident in HBM",
                   "stage_ms": {x: round(v, 3) for x, v in stage_ms.items()},
                   "outside_step": {"generate_s": round(gen_s, 1), "h2d_ms": round(up_ms, 1),
                                    "pack_ms": round(pack_ms, 1)}},
        "roofline": {"kernel": "k_pass1_stream" if occ else "k_pass1_owned", "bound": "hbm",
                     "bytes_per_position": round(bpp, 1), "s": round(s_seen, 4),
                     "frac": round(bpp * owned / (stage_ms["pass1"] / 1000) / 1e9 / HBM_PEAK_GBS, 4),
                     "frac_step": round(bpp * owned / (step_ms / 1000) / 1e9 / HBM_PEAK_GBS, 4)},
        "oracle_check": check,
        "cpu_baseline": cpu,
        "events_per_owned_position": {x: round(v / max(owned, 1), 4) for x, v in st.items()},
    }
    if binned is None or "error" in binned:
        rec["binned_path"] = binned
        return rec
    # the binned path's export equals the table path's (checked every step), which equals the oracle
    # on the sub-shard: the faster of the two is the record, the other its sub-record
    if binned["ms_per_step"] >= rec["ms_per_step"]:
        rec["binned_path"] = binned
        return rec
    table = {x: rec.pop(x) for x in ("value", "ms_per_step", "roofline", "events_per_owned_position")}
    table["stage_ms"] = rec["config"].pop("stage_ms")
    table["step"] = rec["config"].pop("step")
    rec["value"], rec["ms_per_step"] = binned.pop("value"), binned.pop("ms_per_step")
    rec["config"]["path"] = "binned"
    rec["config"]["step"] = binned.pop("step")
    rec["config"]["stage_ms"] = binned.pop("stage_ms")
    rec["config"]["scanned_positions_per_s"] = round(scanned / (rec["ms_per_step"] / 1000), 1)
    rec["config"]["bins"] = binned.pop("bins")
    rec["binned_check"] = binned
    rec["table_path"] = table
    return rec


def run_binned_share(args, dev, packs, sketch, occ, card, p, k, ref_digest, n_rec, owned) -> dict:
    """The human-scale share through the binned path: the same cardinality pass writing the owned
    occurrences, then the stream partitioned into LDS-sized bins (hm_bin_occ) and counted there
    (hm_count_bins; a spilled bin through the table path).  Every step's export must equal the
    table path's (its digest and its record count)."""
    import torch
    from paper_1705_11147_amd import abi, kmer

    g, b = kmer.plan_bins(card.distinct_hi(), card.kept_hi(), p.min_depth == 1)
    if args.share_bins:
        g, b = (int(x) for x in args.share_bins.split(","))
    bc = kmer.BinnedCounter(k, occ.capacity, g, b, min_depth=p.min_depth, n_owners=p.n_owners, owner=p.owner,
                            device=dev)
    out = kmer.Records(int(n_rec * 1.2) + 4096, device=dev)
    log("binned share: 2^%d bins (%d x %d), bins %.1f GB" % (g + b, 1 << g, 1 << b, 2 * bc.capacity * 16 / 1e9))
    stages = ["card", "partition", "count"]
    spilled = [0]

    def step(ev):
        ev[0].record()
        sketch.reset()
        occ.reset()
        for pk in packs:
            sketch.update(pk, occ=occ)
        sketch.summarize(min_depth=p.min_depth)
        ev[1].record()
        bc.bin_occ(occ)
        ev[2].record()
        bc.count(out)
        ev[3].record()
        n_sp = bc.spilled()  # synchronizes; a spilled bin is counted by the table path
        if n_sp:
            spilled[0] += n_sp
            bc.finish(out)

    n_steps = max(1, min(args.steps, 3))
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(n_steps + 1)]
    for s in range(n_steps + 1):  # the first is a warm-up
        step(events[s])
        torch.cuda.synchronize()
        abi.check(bc.status(), "binned human share step")
        same = out.digest_words() == ref_digest and int(out.n_out.item()) == n_rec
        assert same, "the binned share's export differs from the table path's"
        log("binned share step %d of %d done" % (s + 1, n_steps + 1))
    timed = events[1:]
    stage_ms = {x: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in timed])) for i, x in enumerate(stages)}
    step_ms = float(np.mean([ev[0].elapsed_time(ev[len(stages)]) for ev in timed]))
    st = bc.stats()
    return {"value": round(owned / (step_ms / 1000), 1), "ms_per_step": round(step_ms, 3),
            "step": "cardinality pass writing the owned occurrences + partition of the stream into LDS-sized bins "
                    "+ per-bin Bloom filter, table, classification and export in workgroup memory; packed reads "
                    "resident in HBM",
            "stage_ms": {x: round(v, 3) for x, v in stage_ms.items()},
            "bins": {"group_bits": g, "bin_bits": b, "n_bins": 1 << (g + b), "records": st["records"],
                     "spilled_bins": st["spilled_bins"], "spilled": st["spilled"], "deferred": st["deferred"],
                     "keys": st["keys"], "kept": st["kept"], "spilled_records_per_step": spilled[0] // (n_steps + 1)},
            "identical_to_table_path": True}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = the full mid workload)")
    ap.add_argument("--workload", choices=["mid", "mid-heavy", "human-share"], default="mid",
                    help="mid: the headline workload; mid-heavy: mid with 2%% satellite arrays (heavy hitters); "
                         "human-share: one GPU's share of the human-scale run (owner 0 of 16, streamed batches; "
                         "its own JSON line)")
    ap.add_argument("--cpu-sample-reads", type=int, default=2_000_000,
                    help="reads of the headline workload the CPU oracle is timed on (default 10%%)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the oracle comparison of one key shard of the timed export")
    ap.add_argument("--no-probe", action="store_true", help="skip the random-access ceiling probe")
    ap.add_argument("--no-sort", action="store_true", help="skip the key-ordered export measurement")
    ap.add_argument("--bloom-bits", type=float, default=12.0,
                    help="Bloom filter bits per distinct k-mer before rounding the filter to a power of two")
    ap.add_argument("--n-hash", type=int, default=4, help="Bloom filter bits set per k-mer (in one filter word)")
    ap.add_argument("--table-load", type=float, default=0.5,
                    help="design load of the count table (the planned capacity is rounded up to a power of two)")
    ap.add_argument("--separate-bloom", action="store_true",
                    help="a separate Bloom filter instead of the one in the table slots' classification words")
    ap.add_argument("--no-contigs", action="store_true", help="skip the contig generation measurement")
    ap.add_argument("--no-h2d", action="store_true", help="skip the host-to-device copy measurement")
    ap.add_argument("--bypass-diag", action="store_true",
                    help="add the Bloom-bypass diagnostic (one pass into a table sized for every distinct k-mer); "
                         "off by default: it launches the same pass-1 kernel, so a kernel trace of the default run "
                         "holds only the measured step's pass 1")
    ap.add_argument("--no-occ-stream", action="store_true",
                    help="human-share: pass 1 scans the reads with the owner filter instead of reading the owned "
                         "occurrences the cardinality pass wrote")
    ap.add_argument("--no-heavy", action="store_true",
                    help="count heavy hitters through the table instead of workgroup-local counters")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batch-sets", type=int, default=64)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--path", choices=["binned", "table"], default="binned",
                    help="the timed step: the binned path (LDS-sized bins) or the table path (one count table in "
                         "HBM); the other is measured as a sub-record")
    ap.add_argument("--share-bins", default=None, metavar="G,B",
                    help="group and bin bits of the human share's binned path (default: kmer.plan_bins)")
    ap.add_argument("--no-binned-share", action="store_true",
                    help="skip the binned path on the human-scale share (the table path alone)")
    ap.add_argument("--no-binned-sub", action="store_true",
                    help="with --path table: skip the binned path's sub-record")
    ap.add_argument("--no-tiny", action="store_true",
                    help="skip the tiny read set (GPU step, full oracle comparison, oracle on 1 and all threads)")
    ap.add_argument("--no-heavy-workload", action="store_true",
                    help="skip the heavy-hitter comparison on the satellite-rich mid workload")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-pool", type=int, default=12)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-scale", type=float, default=1.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-planners", type=int, default=2, help="jobs planned at once in the continuous run")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-human-share", action="store_true",
                    help="skip one GPU's share of the human-scale run (the human_share sub-record)")
    ap.add_argument("--no-human-oracle", action="store_true",
                    help="human share: skip the oracle check of its sub-shard (about a minute of host work)")
    ap.add_argument("--human-scale", type=float, default=1.0, help="human share: workload scale")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this k-mer analysis build runs on a single MI355X "
              "(no multi-GPU path); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1705_11147_amd import abi, kmer, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    abi.lib()
    if args.workload == "human-share":  # its own JSON line
        hs = run_human_share(args, dev)
        print(json.dumps(dict(hs, n_gpus=1, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="u64",
                              data="synthetic")), flush=True)
        return

    t0 = time.time()
    w = synth.mid(scale=args.scale) if args.workload == "mid" else synth.mid_heavy(scale=args.scale)
    r = w.reads()
    p = w.params
    L, k = r.read_len, p.k
    W = L - k + 1
    positions = r.n_reads * W
    log("workload %s: %d reads x %d bp, %.3g positions (generated in %.1fs)" % (w.name, r.n_reads, L, positions,
                                                                            time.time() - t0))
    ascii = torch.from_numpy(r.ascii).to(dev)
    qual = torch.from_numpy(r.qual).to(dev)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    packed = kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut)
    # sizes from the cardinality pass (HyperLogLog estimate + distinct sample), as the paper sizes
    # its Bloom filter before counting
    sketch = kmer.CardSketch(k, positions, device=dev)
    card = sketch.run([packed], min_depth=p.min_depth)
    abi.check(card.status, "cardinality pass")
    in_table = not args.separate_bloom
    cap, bloom_words, list_cap = kmer.plan_sizes(card, n_hash=args.n_hash, bloom_bits=args.bloom_bits,
                                                 table_load=args.table_load, device=dev, bloom_in_table=in_table)
    log("cardinality pass: %.4g distinct (HLL), %d of %d sampled keys kept (1/2^%d), %d heavy hitters "
        "-> table 2^%d, bloom 2^%d words, list %d" % (card.estimate, card.sampled_kept, card.sampled_distinct,
                                                      card.sample_log2, card.n_heavy, cap.bit_length() - 1,
                                                      bloom_words.bit_length() - 1, list_cap))
    while True:
        kc = kmer.KmerCounter(k, cap, bloom_words, list_cap, n_hash=args.n_hash, min_depth=p.min_depth,
                              bloom_in_table=in_table,
                              heavy=None if args.no_heavy else card, device=dev)
        out = kmer.Records(int(cap * 0.6), device=dev)
        kc.run([packed], out, fused=True)
        rc = kc.status()
        if rc == abi.HM_OK:
            break
        if rc == abi.HM_ECAPACITY:
            st = int(kc.status_buf.item())
            log("capacity retry: status 0x%x" % st)
            if st & abi.HM_ST_TABLE_FULL:
                cap *= 2
            if st & abi.HM_ST_LIST_FULL:
                list_cap = int(list_cap * 1.5)
            del kc, out
            continue
        if rc == abi.HM_EOUTPUT:
            need = int(out.n_out.item())
            out = kmer.Records(int(need * 1.1), device=dev)
            kc.run([packed], out, fused=True)
            abi.check(kc.status(), "k-mer analysis")
            break
        abi.check(rc, "k-mer analysis")
    n_records = int(out.n_out.item())
    n_first = int(kc.list_count.item())
    ref_digest = out.digest_words()
    table_slots = kc.capacity
    bloom = ({"layout": "in table: the home slot's 32-bit classification word", "bits": kc.capacity * 32}
             if kc.bloom_in_table else {"layout": "separate: 64-bit words", "bits": kc.bloom_words * 64})
    bloom.update(n_hash=args.n_hash, bits_per_distinct_kmer=round(bloom["bits"] / card.estimate, 2))
    log("sizes: table 2^%d slots (%.1f GB), bloom %s, list %.2f GB; kept %d, first-occurrence %d" % (
        kc.capacity.bit_length() - 1, kc.capacity * 64 / 1e9,
        "in the table" if kc.bloom_in_table else "%.2f GB" % (kc.bloom_words * 8 / 1e9), list_cap * 17 / 1e9,
        n_records, n_first))

    stages = ["pack", "card", "init", "pass1", "pass2", "classify_export"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        kmer.pack_reads(ascii, qual, read_len=L, qcut=p.qcut, out=packed)
        mark(1)
        sketch.reset()  # the cardinality pass (its summary sized the structures once, before the loop)
        sketch.update(packed)
        sketch.summarize(min_depth=p.min_depth)
        mark(2)
        kc.reset()
        mark(3)
        kc.insert(packed)
        mark(4)
        kc.count()
        mark(5)
        kc.export(out, abi.HM_EXPORT_CLASSIFY)  # depth filter + classification fused into the export sweep
        mark(6)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        step(events[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    abi.check(kc.status(), "k-mer analysis (timed steps)")
    assert out.digest_words() == ref_digest and int(out.n_out.item()) == n_records, "output changed between steps"
    again = sketch.result()
    assert (again.estimate, again.sampled_kept, again.n_heavy) == (card.estimate, card.sampled_kept, card.n_heavy), \
        "cardinality pass changed between steps"

    stage_ms = {name: float(np.mean([events[s][i].elapsed_time(events[s][i + 1]) for s in range(args.steps)]))
                for i, name in enumerate(stages)}
    step_ms = np.array([events[s][0].elapsed_time(events[s][len(stages)]) for s in range(args.steps)])
    step_dist = {"median": round(float(np.median(step_ms)), 3), "p10": round(float(np.percentile(step_ms, 10)), 3),
                 "p90": round(float(np.percentile(step_ms, 90)), 3), "n": int(args.steps)}
    ms_per_step = elapsed * 1000 / args.steps
    value = positions * args.steps / elapsed
    log("stage ms: " + ", ".join("%s %.2f" % kv for kv in stage_ms.items()))

    # roofline of the dominant kernel (pass 1).  Algorithmic bytes per k-mer position of the method
    # (line granular, g = one 64-byte line per random access): (1 + s) random read-modify-writes of
    # a line (a Bloom update for every position, a counter update for the fraction s of positions
    # the filter has seen) and one read-only table probe, (1 + s) * 2g + g, with s = 1 - deferred /
    # positions (the positions counted in pass 1) from the pass's own counters.  Pass 1 does most
    # of this work and pass 2 the rest, so `frac` (over the pass-1 kernel's time) is an upper
    # bound; `frac_counting` prices the same bytes over both passes and `frac_step` over the step.
    st = kc.stats()  # cleared by every step's table init: the last step's counts
    occ, bloom_tests, deferred = st["occurrences"] - st["heavy_local"], st["bloom_tests"], st["deferred"]
    s_seen = 1.0 - deferred / max(st["occurrences"], 1)
    bpp = (1.0 + s_seen) * 2 * LINE + LINE
    alg_bytes = bpp * positions
    achieved = alg_bytes / (stage_ms["pass1"] / 1000) / 1e9
    # the pass's own, smaller model from its event counters: a home line read per occurrence
    # counted through the table, written back when counted in pass 1 (or by the Bloom OR of a
    # deferred occurrence, the filter being in the table; a separate filter's word is one more
    # line read and written), 17 bytes per list entry, the packed reads once
    bloom_bytes = deferred * LINE if kc.bloom_in_table else bloom_tests * 2 * LINE
    own_bytes = occ * LINE + (occ - deferred) * LINE + bloom_bytes + deferred * 17 + 0.5 * r.n_bases
    own_achieved = own_bytes / (stage_ms["pass1"] / 1000) / 1e9
    roofline = {"kernel": "k_pass1_fixed (table probe, Bloom test-and-set, insert/count)", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(os.path.join(ROOT, "profiles", "k_pass1_fixed_mid_k51_traffic.md"))
                if args.scale == 1.0 and args.workload == "mid" else None,
                "bytes_per_position": round(bpp, 2), "s": round(s_seen, 4),
                "model": "(1 + s) * 2g + g bytes per position, g = 64 B, s = 1 - deferred / positions",
                "kernel_ms": round(stage_ms["pass1"], 3),
                "frac_counting": round(alg_bytes / ((stage_ms["pass1"] + stage_ms["pass2"]) / 1000) / 1e9
                                       / HBM_PEAK_GBS, 4),
                "frac_step": round(alg_bytes / (step_dist["median"] / 1000) / 1e9 / HBM_PEAK_GBS, 4),
                "own_model": {"bytes_per_position": round(own_bytes / positions, 2),
                              "achieved_GBps": round(own_achieved, 1),
                              "frac": round(own_achieved / HBM_PEAK_GBS, 4)},
                "events_per_position": {x: round(v / positions, 4) for x, v in st.items()}}
    rates = None
    if not args.no_probe:
        from paper_1705_11147_amd import roofline as ra
        m = ra.measure(kc.capacity * 64, kinds=("load", "atomic_add", "atomic_or_ret", "probe_cas"), n_ops=1 << 28,
                       reps=2, device=dev)
        roofline["measured_random_access"] = {
            "footprint_GB": round(m["footprint_bytes"] / 1e9, 2),
            "load_Gops": round(m["load"]["ops_per_s"] / 1e9, 2),
            "atomic_add_Gops": round(m["atomic_add"]["ops_per_s"] / 1e9, 2),
            "atomic_or_ret_Gops": round(m["atomic_or_ret"]["ops_per_s"] / 1e9, 2),
            "probe_cas_Gops": round(m["probe_cas"]["ops_per_s"] / 1e9, 2),
            "copy_GBps": round(m["copy"]["GBps"], 1)}
        # the same pass priced at the measured rates of its own access kinds, one after another: a hit
        # is a probe + CAS on its line; a Bloom test with the filter in the table a probe + an OR on
        # the probed line (priced as a probe + CAS), with a separate filter a probe that misses + an
        # OR with return on another line; every further table line a probe reaches a load (the first
        # two slots share the home line); an insertion two atomics (key claim, count)
        rate = {x: m[x]["ops_per_s"] for x in ("load", "atomic_add", "atomic_or_ret", "probe_cas")}
        rates = dict(rate, copy_Bps=m["copy"]["GBps"] * 1e9)
        hits = st["hit_first_lookup"]
        inserts = max(occ - hits - deferred, 0)
        bloom_s = (bloom_tests / rate["probe_cas"] if kc.bloom_in_table
                   else bloom_tests / rate["load"] + bloom_tests / rate["atomic_or_ret"])
        model_s = (hits / rate["probe_cas"] + bloom_s + max(st["probe_lines"] - occ, 0) / rate["load"]
                   + 2 * inserts / rate["atomic_add"])
        roofline["measured_ceiling_ms"] = round(model_s * 1000, 2)
        roofline["frac_of_measured_ceiling"] = round(model_s * 1000 / stage_ms["pass1"], 4)
        # random memory requests of pass 1 (from the counters): a 16-byte load per probed slot,
        # an 8-byte load of the second key word per match, Bloom ORs, counting CASes (and the
        # wide atomics when a counter overflows its packed lane)
        reqs = st["probe_slots"] + (occ - deferred) + bloom_tests + st["cas_attempts"] + 2 * st["wide_counts"]
        roofline["pass1_random_requests_Gps"] = round(reqs / (stage_ms["pass1"] / 1000) / 1e9, 2)

    binned, bc, out_b = None, None, None
    if args.path == "binned" or not args.no_binned_sub:
        binned, bc, out_b = run_binned_step(args, dev, log, ascii, qual, packed, sketch, card, positions, L, p, stream,
                                            ref_digest, n_records, bpp)

    sorted_export = None
    if not args.no_sort:
        sorted_export = measure_sorted_export(kc, out, k, n_records, ref_digest, stream, log)
    contigs = None
    if not args.no_contigs:
        contigs = measure_contigs(kc, k, n_records, stream, log, rates=rates)

    h2d = None
    if not args.no_h2d:
        # secondary figure: the same ASCII + Phred handed over from pinned host memory (the boundary
        # takes device buffers, so this copy is never part of `value`)
        pa = torch.empty(r.ascii.size, dtype=torch.uint8, pin_memory=True)
        pq = torch.empty(r.qual.size, dtype=torch.uint8, pin_memory=True)
        pa.numpy()[:] = r.ascii
        pq.numpy()[:] = r.qual
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        ascii.copy_(pa, non_blocking=True)
        qual.copy_(pq, non_blocking=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nbytes = r.ascii.size + r.qual.size
        h2d = {"bytes": int(nbytes), "ms": round(ms, 3), "GBps": round(nbytes / (ms / 1000) / 1e9, 2),
               "kmers_per_s_with_h2d": round(positions / (((binned["step_ms"]["median"] if args.path == "binned"
                                                            else step_dist["median"]) + ms) / 1000), 1)}
        log("h2d: %s" % h2d)
        del pa, pq

    bypass = None
    if args.bypass_diag:
        # diagnostic: the paper's pre-Bloom scheme, every occurrence counted in one pass into a table sized
        # for every distinct k-mer (about 4x the Bloom design's table); same digest required
        bcap = kmer.next_pow2(int(card.estimate / 0.45))
        kb = kmer.KmerCounter(k, bcap, 1, 0, min_depth=p.min_depth, flags=abi.HM_BLOOM_BYPASS, device=dev)
        ob = kmer.Records(int(n_records * 1.05), device=dev)
        kb.run([packed], ob, fused=True)  # warm-up
        abi.check(kb.status(), "bypass diagnostic")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        kb.reset()
        ev[1].record(stream)
        kb.insert(packed)
        ev[2].record(stream)
        kb.count()
        ev[3].record(stream)
        kb.export(ob, abi.HM_EXPORT_CLASSIFY)
        ev[4].record(stream)
        torch.cuda.synchronize()
        abi.check(kb.status(), "bypass diagnostic")
        same = ob.digest_words() == ref_digest and int(ob.n_out.item()) == n_records
        bst = kb.stats()
        bms = [ev[i].elapsed_time(ev[i + 1]) for i in range(4)]
        bypass = {"table_slots": kb.capacity, "table_GB": round(kb.capacity * 64 / 1e9, 1),
                  "init_ms": round(bms[0], 3), "pass1_ms": round(bms[1], 3), "pass2_ms": round(bms[2], 3),
                  "export_ms": round(bms[3], 3), "total_ms": round(sum(bms), 3), "same_digest": same,
                  "events_per_position": {x: round(v / positions, 4) for x, v in bst.items()}}
        log("bloom-bypass diagnostic: %s" % bypass)
        assert same, "bypass diagnostic changed the table"
        del kb, ob
        torch.cuda.empty_cache()

    # the timed export against the oracle: every record of one key shard (1/64 of the keys, by a
    # hash independent of the table layout), field by field
    oracle_check = None
    threads = host_threads()
    if not args.no_oracle_check:
        import oracle
        n_shards, shard = 64, 5
        t1 = time.perf_counter()
        timed = out_b if args.path == "binned" else out  # the export of the timed steps
        hk = timed.key_hi[:n_records].cpu().numpy().view(np.uint64)
        lk = timed.key_lo[:n_records].cpu().numpy().view(np.uint64)
        idx = np.nonzero(oracle.shard_of(hk, lk, n_shards) == shard)[0]
        del hk, lk
        got = device_rows(timed, torch.from_numpy(idx).to(dev))
        exp = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=p.qcut, min_depth=p.min_depth, n_shards=n_shards,
                         shard=shard, n_threads=threads, sort_count=True)
        same = same_records(got, exp)
        oracle_check = {"shard": "%d of %d" % (shard, n_shards), "records": len(got["count"]),
                        "oracle_records": len(exp["count"]), "oracle_identical": same,
                        "oracle_positions": exp["positions"], "s": round(time.perf_counter() - t1, 1)}
        log("oracle check of the timed export: %s" % oracle_check)
        assert same and exp["positions"] == positions, "the timed export disagrees with the oracle on its shard"
        del got, exp

    cpu = None
    if not args.no_cpu:
        import oracle
        # the oracle timed on the first cpu_sample_reads reads (sort-counted, every host core), and the
        # GPU path on the same sample, which must give the same table record by record
        n_cpu = min(args.cpu_sample_reads, r.n_reads)
        sub_a = r.ascii[: n_cpu * L]
        sub_q = r.qual[: n_cpu * L]
        off = np.arange(n_cpu + 1, dtype=np.int64) * L
        res = oracle.run(sub_a, sub_q, off, k, qcut=p.qcut, min_depth=p.min_depth, n_threads=threads,
                         sort_count=True)
        del kc, out, bc, out_b
        torch.cuda.empty_cache()
        g = kmer.analyze(sub_a, sub_q, k, read_len=L, qcut=p.qcut, min_depth=p.min_depth,
                         export_flags=abi.HM_EXPORT_SORTED, fused=True, binned=args.path == "binned", device=dev)
        same = same_records(g, res)
        assert same, "the GPU table of the CPU-baseline sample disagrees with the oracle"
        cpu = {"value": round(n_cpu * W / res["seconds"], 1), "unit": "k-mers/s", "cores": threads,
               "kind": "oracle",
               "sample": "first %d reads (%d positions, %.0f%% of the workload), sort-counted on %d threads, %.1fs; "
                         "the GPU's table of the same sample (%s path) is identical (%d records); %s" % (
                             n_cpu, n_cpu * W, 100.0 * n_cpu / r.n_reads, threads, res["seconds"], args.path,
                             len(res["count"]), cpu_model())}
        log("cpu baseline: %s" % cpu)
        del g, res
        kc = out = bc = out_b = None

    del kc, out, bc, out_b, packed, ascii, qual
    torch.cuda.empty_cache()
    tiny = None
    if not args.no_tiny:
        tiny = run_tiny(args, dev, log)
        torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        batched = run_batched(args, dev, log)
    heavy = None
    if not args.no_heavy_workload:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        heavy = run_heavy(args, dev, log)
    serving = None
    if not args.no_serving:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        serving = run_serving(args, dev, log)
    human = None
    if not args.no_human_share:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        human = run_human_share(args, dev)

    cardinality = {"hll_estimate": round(card.estimate, 1), "hll_p": card.hll_p, "sampled_kept": card.sampled_kept,
                   "sample_log2": card.sample_log2, "kept_estimate": card.sampled_kept << card.sample_log2,
                   "heavy_hitters": card.n_heavy}
    table_step = "pack+cardinality+init+pass1+pass2+(classify fused into export), inputs resident in HBM"
    table_path = {"value": round(value, 1), "ms_per_step": round(ms_per_step, 3), "table_slots": table_slots,
                  "bloom": bloom, "step": table_step, "stage_ms": {x: round(v, 3) for x, v in stage_ms.items()},
                  "step_ms": step_dist, "roofline": roofline}
    config = {"workload": w.name, "genome_bp": int(w.meta["G"]), "reads": r.n_reads, "read_len": L, "k": k,
              "qcut": p.qcut, "min_depth": p.min_depth, "positions": positions, "kept_kmers": n_records,
              "cardinality": cardinality}
    if args.path == "binned":
        head = binned
        config.update(path="binned", step="pack+cardinality+partition into LDS-sized bins+per-bin Bloom filter, "
                                           "table, classification and export in workgroup memory (spilled bins "
                                           "through the table path), inputs resident in HBM",
                      bins=binned["bins"], stage_ms=binned["stage_ms"], step_ms=binned["step_ms"])
        sub = {"table_path": table_path}
    else:
        head = dict(table_path, value=value, ms_per_step=ms_per_step)
        config.update(path="table", table_slots=table_slots, bloom=bloom, step=table_step,
                      stage_ms=table_path["stage_ms"], step_ms=step_dist)
        sub = {"binned_path": {x: binned[x] for x in ("value", "ms_per_step", "stage_ms", "step_ms", "bins",
                                                      "roofline")} if binned else None}
    line = {
        "metric": METRIC, "value": round(head["value"], 1), "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": config,
        "roofline": head["roofline"],
        **sub,
        "oracle_check": oracle_check,
        "cpu_baseline": cpu,
        "sorted_export": sorted_export,
        "contigs": contigs,
        "h2d": h2d,
        "bloom_bypass_diagnostic": bypass,
        "tiny": tiny,
        "batched": batched,
        "heavy_hitters": heavy,
        "serving": serving,
        "human_share": human,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
