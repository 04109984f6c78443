"""Serving loop for k-mer analysis jobs: continuous batching on one GPU.

Jobs arrive open-loop (e.g. Poisson).  The scheduler admits them in arrival
order as soon as a slot is free and the job's HBM footprint fits the free
budget.  It does not wait for the running jobs to drain: a job that arrives
while others are on the GPU starts as soon as a slot and memory free up, and
its work overlaps theirs on the device.  Each admitted job runs the whole
path on its own HIP stream:

    pinned host -> HBM copy -> pack -> init -> pass 1 -> pass 2 -> export (classifying inline)

Its table and export stay device-resident until the job completes.  Latency
is completion time minus arrival time.  The scheduler's thread never waits
on a stream: a job's status word, record count and digest (and a plan's
summary) are copied into pinned host memory on the job's own stream ahead
of the event it polls.  A blocking read would wait behind the other jobs'
kernels, which hold every compute unit while they run, and the scheduler
could neither admit jobs nor start their copies meanwhile.

A backend with `plans` set (and `plan`, `planned`, `finish_plan`, `discard`,
`plan_footprint`)
sizes each job the way the paper sizes its Bloom filter: before admission the
job at the head of the queue is copied to the device, packed and run through
the cardinality pass (HyperLogLog estimate and distinct sample) on its own
stream, holding only those buffers; its exact footprint then decides when it
is admitted.  Up to `max_planning` jobs plan at once, also while every slot
is busy, and planned jobs keep FIFO order.

The scheduler is independent of the device: `GpuBackend` runs jobs through
the C ABI, and tests drive the same scheduler with a fake backend and a
virtual clock.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    id: int
    arrival: float                 # seconds since the start of the run
    n_bases: int
    read_len: int
    distinct_est: float            # size hints (k-mers expected distinct / kept)
    kept_est: float
    payload: object = None         # backend-specific (host tensors for the GPU backend)
    meta: dict = field(default_factory=dict)


@dataclass
class Record:
    job: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    status: int = 0
    retries: int = 0
    result: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep(self, dt: float):
        if dt > 0:
            time.sleep(dt)


class Scheduler:
    """FIFO admission by HBM footprint into at most `max_slots` concurrent jobs."""

    def __init__(self, backend, budget_bytes: int, max_slots: int, poll_s: float = 0.0005, max_planning: int = 2,
                 plan_while_busy: bool = True):
        """max_planning: jobs planned at once (in arrival order).  plan_while_busy: plan also while
        every slot is busy, so that the next job is ready when a slot frees (else a job is planned
        only once a slot is free and no planned job waits: nothing overlaps a running job)."""
        self.backend = backend
        # never more than the backend's own memory, if it states it
        self.budget = min(int(budget_bytes), int(getattr(backend, "capacity_bytes", budget_bytes)))
        self.max_slots = int(max_slots)
        self.poll_s = poll_s
        self.max_planning = max(1, int(max_planning))
        self.plan_while_busy = bool(plan_while_busy)
        self.trace = []  # (time, queued, running, bytes in use)

    def run(self, jobs: list[Job], clock=None, max_retries: int = 3) -> list[Record]:
        clock = clock or WallClock()
        be = self.backend
        planner = bool(getattr(be, "plans", False))
        first_need = be.plan_footprint if planner else be.footprint
        # placement hooks of a backend whose memory can fragment (else the byte budget decides alone)
        can_plan = getattr(be, "can_plan", lambda j, then=None: True)
        can_start = getattr(be, "can_start", lambda j, h=None: True)
        order = sorted(range(len(jobs)), key=lambda i: jobs[i].arrival)
        recs = {j.id: Record(j.id, j.arrival) for j in jobs}
        for j in jobs:
            if first_need(j) > self.budget:
                raise ValueError("job %d needs %d bytes, more than the whole budget %d" % (
                    j.id, first_need(j), self.budget))
        nxt = 0                      # next job (in arrival order) not yet queued
        queue: list[Job] = []
        running = {}                 # job id -> (handle, bytes)
        used = 0
        planning = []                # [job, plan handle, bytes held] of the jobs being planned, oldest first
        ready = None                 # (job, plan handle, bytes held): planned, waiting for admission
        replanned = {}               # job id -> plans given back because the job could not be placed
        while nxt < len(order) or queue or running or planning or ready:
            now = clock.now()
            while nxt < len(order) and jobs[order[nxt]].arrival <= now:
                queue.append(jobs[order[nxt]])
                nxt += 1
            # completions first: they free slots and memory for admissions
            for jid in list(running):
                h, b = running[jid]
                if be.poll(h):
                    status, result = be.finish(h)
                    used -= b
                    del running[jid]
                    r = recs[jid]
                    if status == "retry" and r.retries < max_retries and first_need(result) <= self.budget:
                        r.retries += 1
                        queue.insert(0, result)  # the backend returns the resized job
                        continue
                    if status == "retry":
                        status, result = "capacity", None
                    r.done = clock.now()
                    r.status = 0 if status == "ok" else status
                    r.result = result
            # the oldest plan becomes ready when it is done (later ones wait their turn: FIFO)
            if ready is None and planning and be.planned(planning[0][1]):
                j, h, pb = planning.pop(0)
                ready = (be.finish_plan(h), h, pb)
            # admission: FIFO, head of line waits for memory
            while len(running) < self.max_slots:
                if planner:
                    if ready is None:
                        break
                    j, h, pb = ready
                    b = be.footprint(j)
                    if b > self.budget:  # the planned job cannot fit at all
                        be.discard(h)
                        used -= pb
                        ready = None
                        recs[j.id].done = clock.now()
                        recs[j.id].status = "capacity"
                        continue
                    if used - pb + b > self.budget or not can_start(j, h):
                        break
                    ready = None
                    running[j.id] = (be.start(j, h), b)
                    used += b - pb
                    continue
                if not queue:
                    break
                j = queue[0]
                b = be.footprint(j)
                if used + b > self.budget or not can_start(j):
                    break
                queue.pop(0)
                if np.isnan(recs[j.id].admitted):
                    recs[j.id].admitted = clock.now()
                running[j.id] = (be.start(j), b)
                used += b
            if planner and (self.plan_while_busy or (len(running) < self.max_slots and ready is None)):
                # plan ahead, in arrival order, while the budget holds the plans' buffers and still
                # leaves the ready job room to be admitted (a plan must never keep it waiting)
                held = be.footprint(ready[0]) - ready[2] if ready is not None else 0
                while len(planning) < self.max_planning and queue:
                    j = queue[0]
                    pb = be.plan_footprint(j)
                    if used + max(held, 0) + pb > self.budget or not can_plan(j, ready[0] if ready else None):
                        break
                    queue.pop(0)
                    if np.isnan(recs[j.id].admitted):
                        recs[j.id].admitted = clock.now()
                    planning.append([j, be.plan(j), pb])
                    used += pb
                # nothing running and the ready job does not fit beside the later plans' buffers:
                # give back the newest finished plan (its job goes back to the queue's front); with
                # no later plan, a ready job that cannot be placed alone gives back its own plan and
                # is planned again into memory that is then free
                if ready is not None and not running:
                    rj, rh, rpb = ready
                    blocked = used - rpb + be.footprint(rj) > self.budget or not can_start(rj, rh)
                    if blocked and planning and be.planned(planning[-1][1]):
                        j, h, pb = planning.pop()
                        be.discard(h)
                        used -= pb
                        queue.insert(0, j)
                    elif blocked and not planning:
                        be.discard(rh)
                        used -= rpb
                        ready = None
                        replanned[rj.id] = replanned.get(rj.id, 0) + 1
                        if replanned[rj.id] > 1:  # blocked alone in empty memory: it cannot fit
                            recs[rj.id].done = clock.now()
                            recs[rj.id].status = "capacity"
                        else:
                            meta = {x: v for x, v in rj.meta.items() if x not in ("plan", "card")}
                            queue.insert(0, Job(rj.id, rj.arrival, rj.n_bases, rj.read_len, rj.distinct_est,
                                                rj.kept_est, rj.payload, meta))
            self.trace.append((now, len(queue), len(running), used))
            if running or queue or planning or ready:
                clock.sleep(self.poll_s)
            elif nxt < len(order):
                clock.sleep(max(0.0, jobs[order[nxt]].arrival - clock.now()))
        return [recs[j.id] for j in jobs]


def summarize(recs: list[Record], positions: dict, trace=None) -> dict:
    """Latency percentiles, throughput over the makespan, offered load."""
    lat = np.array([r.latency for r in recs])
    arr = np.array([r.arrival for r in recs])
    done = np.array([r.done for r in recs])
    total_pos = float(sum(positions[r.job] for r in recs))
    makespan = float(done.max() - arr.min())
    span_arr = float(arr.max() - arr.min()) or 1e-9
    out = {"jobs": len(recs), "p50_ms": float(np.percentile(lat, 50) * 1000),
           "p99_ms": float(np.percentile(lat, 99) * 1000), "max_ms": float(lat.max() * 1000),
           "mean_ms": float(lat.mean() * 1000), "kmers_per_s": total_pos / makespan, "makespan_s": makespan,
           "offered_kmers_per_s": total_pos / span_arr, "offered_jobs_per_s": (len(recs) - 1) / span_arr,
           "retries": int(sum(r.retries for r in recs)), "failed": int(sum(1 for r in recs if r.status != 0))}
    if trace:
        t = np.array(trace, dtype=np.float64)
        if len(t) > 1:
            w = np.diff(t[:, 0])
            out["mean_in_flight"] = float((t[:-1, 2] * w).sum() / max(w.sum(), 1e-9))
            out["mean_queued"] = float((t[:-1, 1] * w).sum() / max(w.sum(), 1e-9))
            out["max_queued"] = int(t[:, 1].max())
    return out


class GpuBackend:
    """Runs each job through the C ABI on its own HIP stream.  With plan=True
    (default) each job is sized by a cardinality pass before admission; with
    plan=False by the job's own size hints (distinct_est, kept_est).

    Device memory: one arena of `memory_bytes`, reserved at construction
    (give the scheduler the same budget).  A job holds three slabs of it:
    its ASCII and quality bytes with the cardinality pass's state (from the
    plan until the plan has finished: the packed reads replace them), its
    packed reads (until the job completes) and its table, list and output
    (from admission until the job completes).  The scheduler asks
    can_plan / can_start whether the slabs can be placed, besides its byte
    budget."""

    def __init__(self, k: int, qcut: int = 20, min_depth: int = 2, table_load: float = 0.45, bloom_bits: float = 12.0,
                 n_hash: int = 4, device="cuda", plan: bool = True, keep_records: bool = False,
                 memory_bytes: int = 8 << 30):
        """keep_records: copy every finished job's records to the host, sorted by key
        (`records[job id]`), besides the count and digest each result holds."""
        import torch
        from .arena import DeviceArena
        self.torch = torch
        self.keep_records = keep_records
        self.records = {}
        self.device = torch.device(device)
        self.k, self.qcut, self.min_depth = k, qcut, min_depth
        self.table_load, self.bloom_bits, self.n_hash = table_load, bloom_bits, n_hash
        self._streams = []
        self.plans = plan  # the scheduler plans jobs (cardinality pass) before admission
        self.arena = DeviceArena(memory_bytes, self.device)
        self.capacity_bytes = self.arena.size

    # ---- sizes
    def _hint_sizes(self, j: Job):
        from .kmer import next_pow2
        cap = next_pow2(max(1024, int(j.meta.get("kept", j.kept_est) / self.table_load)))
        bw = next_pow2(max(64, int(j.distinct_est * self.bloom_bits / 64)))
        lcap = int(j.meta.get("list", j.distinct_est * 1.2)) + (1 << 20) + 4 * 8192 * 255
        ocap = int(min(cap, j.meta.get("out", j.meta.get("kept", j.kept_est) * 1.3 + 1024)))
        return cap, bw, lcap, ocap

    def sizes(self, j: Job):
        return j.meta["plan"] if "plan" in j.meta else self._hint_sizes(j)

    def _slab_bytes(self, j: Job) -> tuple[int, int]:
        """(bytes of the slab with ASCII, quality and the cardinality state, bytes of the packed reads)."""
        from .kmer import CardSketch, packed_bytes, tensor_bytes
        reads = 2 * tensor_bytes(j.n_bases, 1)
        if self.plans:
            reads += CardSketch.bytes_for(j.n_bases)
        return reads, packed_bytes(j.n_bases)

    def _count_bytes(self, j: Job) -> int:
        from .kmer import KmerCounter, Records
        cap, bw, lcap, ocap = self.sizes(j)
        card = j.meta.get("card")
        n_heavy = 0 if card is None else min(len(card.heavy_hi), self._max_heavy())
        return (KmerCounter.bytes_for(cap, bw, lcap, n_heavy, min_depth=self.min_depth)
                + Records.bytes_for(ocap))

    @staticmethod
    def _max_heavy() -> int:
        from . import abi
        return abi.HM_MAX_HEAVY

    def plan_footprint(self, j: Job) -> int:
        return sum(self._slab_bytes(j))

    def footprint(self, j: Job) -> int:
        """Bytes the job holds while it counts (a planned job no longer holds its ASCII and quality)."""
        reads, packed = self._slab_bytes(j)
        return (packed if "plan" in j.meta else reads + packed) + self._count_bytes(j)

    def can_plan(self, j: Job, then: Job | None = None) -> bool:
        """Whether j's plan slabs can be placed now, and still leave room for the counting slab
        of `then` (the planned job waiting for admission)."""
        need = list(self._slab_bytes(j))
        if then is not None:
            need.append(self._count_bytes(then))
        return self.arena.fits(need)

    def can_start(self, j: Job, plan_handle=None) -> bool:
        need = [self._count_bytes(j)]
        if plan_handle is None:
            need = list(self._slab_bytes(j)) + need
        return self.arena.fits(need)

    def _stream(self):
        return self._streams.pop() if self._streams else self.torch.cuda.Stream(device=self.device)

    # ---- planning: reads to the device, pack, cardinality pass
    def _upload(self, j: Job, st, slabs):
        """Copy the job's reads in and pack them, on stream st, into the two slabs (reads, packed)."""
        from . import kmer
        torch = self.torch
        ascii_h, qual_h = j.payload
        reads, packed_slab = slabs
        with torch.cuda.stream(st):
            a = reads.empty(j.n_bases, torch.uint8)[:j.n_bases]
            q = reads.empty(j.n_bases, torch.uint8)[:j.n_bases]
            a.copy_(ascii_h, non_blocking=True)
            q.copy_(qual_h, non_blocking=True)
            packed = kmer.pack_reads(a, q, read_len=j.read_len, qcut=self.qcut, stream=st,
                                     out=kmer.new_packed(j.n_bases, self.device, packed_slab))
        return packed

    def _slabs(self, j: Job):
        from .arena import Slab
        reads_b, packed_b = self._slab_bytes(j)
        packed = Slab(self.arena, packed_b)
        try:
            reads = Slab(self.arena, reads_b, high=True)  # short-lived: the high end
        except MemoryError:
            packed.release()
            raise
        return reads, packed

    def plan(self, j: Job):
        from . import kmer
        torch = self.torch
        st = self._stream()
        slabs = self._slabs(j)
        packed = self._upload(j, st, slabs)
        with torch.cuda.stream(st):
            sk = kmer.CardSketch(self.k, j.n_bases, device=self.device, alloc=slabs[0])
            sk.reset(st)
            sk.update(packed, st)
            sk.summarize(min_depth=self.min_depth, stream=st)
            fetched = sk.fetch(st)  # read after the event: the scheduler never blocks on a stream
            ev = torch.cuda.Event()
            ev.record(st)
        return {"job": j, "stream": st, "event": ev, "sketch": sk, "fetched": fetched, "packed": packed,
                "slabs": list(slabs)}

    def planned(self, h) -> bool:
        return h["event"].query()

    def finish_plan(self, h) -> Job:
        """The planned job, with table / filter / list / output sizes from its cardinality pass
        (doubled per earlier capacity retry).  The plan's event has completed, so the slab of
        ASCII, quality and cardinality state is released here."""
        from . import kmer
        j = h["job"]
        card = h.pop("sketch").decode(h.pop("fetched"))
        h["slabs"][0].release()
        cap, bw, lcap = kmer.plan_sizes(card, n_hash=self.n_hash, bloom_bits=self.bloom_bits,
                                        table_load=self.table_load, device=self.device)
        cap *= j.meta.get("grow_table", 1)
        lcap *= j.meta.get("grow_list", 1)
        ocap = int(min(cap, card.kept_hi() * 1.3 + 1024) * j.meta.get("grow_out", 1))
        meta = dict(j.meta, plan=(cap, bw, lcap, ocap), card=card)
        return Job(j.id, j.arrival, j.n_bases, j.read_len, j.distinct_est, j.kept_est, j.payload, meta)

    def discard(self, h):
        """Give back a plan (finished, or not yet started counting)."""
        if "event" in h:
            h["event"].synchronize()
        for sl in h.get("slabs", ()):
            sl.release()
        if "stream" in h:
            self._streams.append(h["stream"])
        h.clear()

    # ---- the counting passes
    def start(self, j: Job, plan_handle=None):
        from . import kmer
        from .arena import Slab
        torch = self.torch
        cap, bw, lcap, ocap = self.sizes(j)
        if plan_handle is not None:
            st, packed, slabs = plan_handle["stream"], plan_handle["packed"], plan_handle["slabs"]
        else:
            st = self._stream()
            slabs = list(self._slabs(j))
            packed = self._upload(j, st, slabs)
        count = Slab(self.arena, self._count_bytes(j))
        slabs.append(count)
        with torch.cuda.stream(st):
            kc = kmer.KmerCounter(self.k, cap, bw, lcap, n_hash=self.n_hash, min_depth=self.min_depth,
                                  heavy=j.meta.get("card"), device=self.device, alloc=count)
            out = kmer.Records(ocap, device=self.device, alloc=count)
            kc.run([packed], out, stream=st, fused=True)
            fetched = (kc.fetch_status(st),) + out.fetch_summary(st)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"job": j, "stream": st, "event": ev, "kc": kc, "out": out, "fetched": fetched, "slabs": slabs}

    def poll(self, h) -> bool:
        return h["event"].query()

    def finish(self, h):
        from . import abi
        kc, out, st, j = h["kc"], h["out"], h["stream"], h["job"]
        word, n_out, digest = h["fetched"]  # pinned host copies: the job's event has completed
        rc = kc.status_code(word)
        result = None
        status = "ok"
        if rc == abi.HM_OK:
            result = {"n_out": int(n_out[0]), "digest": out.digest_words((n_out, digest))}
            if self.keep_records:
                self.records[j.id] = out.to_numpy(int(n_out[0]))
        elif rc in (abi.HM_ECAPACITY, abi.HM_EOUTPUT):
            # too small for this job: rerun from scratch with the structure that overflowed doubled
            s = int(word[0]) & 0xFFFFFFFF
            meta = {x: v for x, v in j.meta.items() if x not in ("plan", "card")}
            if s & abi.HM_ST_TABLE_FULL:
                meta["kept"] = 2 * meta.get("kept", j.kept_est)
                meta["grow_table"] = 2 * meta.get("grow_table", 1)
            if s & abi.HM_ST_LIST_FULL:
                meta["list"] = 2 * meta.get("list", j.distinct_est * 1.2)
                meta["grow_list"] = 2 * meta.get("grow_list", 1)
            if rc == abi.HM_EOUTPUT:
                meta["out"] = int(int(n_out[0]) * 1.1) + 1024
                meta["grow_out"] = 2 * meta.get("grow_out", 1)
            status, result = "retry", Job(j.id, j.arrival, j.n_bases, j.read_len, j.distinct_est, j.kept_est,
                                          j.payload, meta)
        else:
            status = rc
        for sl in h["slabs"]:  # the job's work on the device has completed
            sl.release()
        h.clear()
        self._streams.append(st)
        return status, result


def make_jobs(pool, n_jobs: int, rate: float, seed: int = 170511151, pin: bool = True):
    """An open-loop Poisson stream of `n_jobs` jobs at `rate` jobs/s whose
    payloads cycle through `pool` (list of synth Workloads), each read once
    into (pinned) host tensors."""
    import torch
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    payloads = []
    for w in pool:
        r = w.reads()
        a = torch.from_numpy(r.ascii)
        q = torch.from_numpy(r.qual)
        if pin:
            a, q = a.pin_memory(), q.pin_memory()
        d, kept = w.size_estimates()
        payloads.append((a, q, r.n_bases, r.read_len, d, kept, w.positions))
    jobs, positions = [], {}
    for i in range(n_jobs):
        a, q, nb, L, d, kept, pos = payloads[i % len(payloads)]
        jobs.append(Job(i, float(arrivals[i]), nb, L, d, kept, (a, q), {"pool": i % len(payloads)}))
        positions[i] = pos
    return jobs, positions
