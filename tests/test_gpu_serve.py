"""Serving on the GPU: every job's result is the same alone and in the mix
(tolerance 0: integer output), and equals the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, synth
from paper_1705_11147_amd.serve import GpuBackend, Scheduler, make_jobs, summarize
from tests.util import assert_tables_equal, table_digest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def test_alone_equals_in_mix_equals_oracle():
    _, builders = synth.serving_jobs(n_jobs=5, scale=0.005)
    pool = [b() for b in builders]
    jobs, positions = make_jobs(pool, n_jobs=10, rate=400.0)
    be = GpuBackend(51)
    mix = Scheduler(be, budget_bytes=8 << 30, max_slots=4).run(jobs)
    assert all(r.status == 0 for r in mix)
    assert all(r.retries == 0 for r in mix)  # planned from a cardinality pass: no job had to grow
    s = summarize(mix, positions)
    assert s["jobs"] == 10 and s["failed"] == 0
    # the same job twice in the stream, and alone on an idle GPU
    for r in mix:
        twin = [x for x in mix if x.job % 5 == r.job % 5]
        assert all(x.result == r.result for x in twin)
    for p in range(5):
        alone = Scheduler(GpuBackend(51), budget_bytes=8 << 30, max_slots=1).run([jobs[p]])
        assert alone[0].result == mix[p].result, p
    for p in (0, 3):
        w = pool[p]
        rd = w.reads()
        exp = oracle.run(rd.ascii, rd.qual, rd.offsets(), 51, n_threads=4)
        assert mix[p].result["n_out"] == len(exp["count"])
        assert mix[p].result["digest"] == table_digest(exp)


def test_sixteen_jobs_record_by_record():
    """16 seeded jobs of the serving recipe (hexaploid-like genomes, distinct sizes) served together
    with continuous batching: every job's records equal the oracle's field by field, and equal the
    records of the same job served alone."""
    n = 16
    _, builders = synth.serving_jobs(n_jobs=n, scale=0.004)
    pool = [b() for b in builders]
    jobs, positions = make_jobs(pool, n_jobs=n, rate=400.0)
    mix_be = GpuBackend(51, keep_records=True)
    mix = Scheduler(mix_be, budget_bytes=8 << 30, max_slots=4).run(jobs)
    assert all(r.status == 0 for r in mix) and len(mix_be.records) == n
    s = summarize(mix, positions)
    assert s["jobs"] == n and s["failed"] == 0
    alone_be = GpuBackend(51, keep_records=True)
    for j in jobs:
        Scheduler(alone_be, budget_bytes=8 << 30, max_slots=1).run([j])
    for j, w in zip(jobs, pool):
        rd = w.reads()
        exp = oracle.run(rd.ascii, rd.qual, rd.offsets(), 51, n_threads=8, sort_count=True)
        assert len(exp["count"]) > 100
        assert_tables_equal(mix_be.records[j.id], exp, "job %d in the mix vs the oracle" % j.id)
        assert_tables_equal(alone_be.records[j.id], mix_be.records[j.id], "job %d alone vs in the mix" % j.id)


def test_capacity_retry_in_serving():
    _, builders = synth.serving_jobs(n_jobs=2, scale=0.005)
    pool = [b() for b in builders]
    jobs, _ = make_jobs(pool, n_jobs=2, rate=100.0)
    for j in jobs:  # far too small a table and filter: the server must resize and rerun
        j.kept_est = 100.0
        j.distinct_est = 100.0  # (the filter in the table would otherwise size the table from it)
    # sized from the (wrong) hints instead of a cardinality pass
    recs = Scheduler(GpuBackend(51, plan=False), budget_bytes=8 << 30, max_slots=2).run(jobs, max_retries=20)
    assert all(r.status == 0 and r.retries > 0 for r in recs)
    rd = pool[1].reads()
    exp = oracle.run(rd.ascii, rd.qual, rd.offsets(), 51)
    assert recs[1].result["digest"] == table_digest(exp)


def test_planned_and_hinted_sizing_agree():
    """A job planned from its cardinality pass and the same job sized from hints give the same
    result; the planned job's structures are not larger than needed by more than the plan's margins."""
    _, builders = synth.serving_jobs(n_jobs=3, scale=0.005)
    pool = [b() for b in builders]
    jobs, _ = make_jobs(pool, n_jobs=3, rate=100.0)
    planned = Scheduler(GpuBackend(51), budget_bytes=8 << 30, max_slots=2).run(jobs)
    hinted = Scheduler(GpuBackend(51, plan=False), budget_bytes=8 << 30, max_slots=2).run(jobs, max_retries=20)
    assert [r.result for r in planned] == [r.result for r in hinted]
    assert all(r.status == 0 for r in planned)


def test_tight_arena_waits_and_agrees():
    """The same job stream through an arena barely larger than what one job at a time needs:
    jobs wait for room (and may be planned again when their slabs cannot be placed), every
    result equals the one from a roomy arena, nothing spills, and the arena is empty at the end."""
    _, builders = synth.serving_jobs(n_jobs=6, scale=0.005)
    pool = [b() for b in builders]
    jobs, _ = make_jobs(pool, n_jobs=12, rate=400.0)
    roomy = GpuBackend(51)
    ref = Scheduler(roomy, budget_bytes=8 << 30, max_slots=1, max_planning=1, plan_while_busy=False).run(jobs)
    assert all(r.status == 0 for r in ref)
    one_at_a_time = roomy.arena.peak
    tight = GpuBackend(51, memory_bytes=int(one_at_a_time * 1.3))
    sch = Scheduler(tight, budget_bytes=8 << 30, max_slots=4, max_planning=2)
    assert sch.budget == tight.arena.size
    got = sch.run(jobs)
    assert [r.result for r in got] == [r.result for r in ref]
    assert tight.arena.used == 0 and tight.arena.spills == 0 and roomy.arena.spills == 0
    assert tight.arena.peak <= tight.arena.size


def test_degenerate_jobs_in_the_mix():
    """A job with no reads and a job whose reads are shorter than k, served among ordinary jobs:
    both complete with the oracle's empty table, and the ordinary jobs' results are the ones they
    get without them."""
    from paper_1705_11147_amd.serve import Job
    _, builders = synth.serving_jobs(n_jobs=3, scale=0.003)
    pool = [b() for b in builders]
    jobs, _ = make_jobs(pool, n_jobs=3, rate=400.0)
    ref = Scheduler(GpuBackend(51), budget_bytes=8 << 30, max_slots=4).run(jobs)
    assert all(r.status == 0 for r in ref)
    rng = np.random.default_rng(3)
    short_a = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 40 * 10)]
    short_q = np.full(40 * 10, 40, np.uint8)
    pin = lambda x: torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
    empty = Job(100, 0.001, 0, 150, 1.0, 1.0, (pin(np.zeros(0, np.uint8)), pin(np.zeros(0, np.uint8))), {})
    short = Job(101, 0.002, 400, 40, 1.0, 1.0, (pin(short_a), pin(short_q)), {})
    be = GpuBackend(51, keep_records=True)
    got = Scheduler(be, budget_bytes=8 << 30, max_slots=4).run(jobs + [empty, short])
    assert [r.status for r in got] == [0] * 5
    assert [r.result for r in got[:3]] == [r.result for r in ref]
    off = np.arange(0, 401, 40, dtype=np.int64)
    exp = oracle.run(short_a, short_q, off, 51)
    assert len(exp["count"]) == 0
    for r in got[3:]:
        assert r.result["n_out"] == 0
        assert len(be.records[r.job]["count"]) == 0
    assert be.arena.used == 0 and be.arena.spills == 0
