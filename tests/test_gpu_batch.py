"""Batched persistent form against the plain per-set path and the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, synth
from paper_1705_11147_amd.batch import Batch, SetSpec, Tuning
from tests.util import assert_tables_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def make_specs(workloads):
    specs, host = [], []
    for w in workloads:
        r = w.reads()
        d, kept = w.size_estimates()
        specs.append(SetSpec(torch.from_numpy(r.ascii).cuda(), torch.from_numpy(r.qual).cuda(), r.read_len, d, kept))
        host.append(r)
    return specs, host


def oracle_table(r, k):
    return oracle.run(r.ascii, r.qual, r.offsets(), k, n_threads=4)


@pytest.mark.parametrize("k", [31, 51])
def test_batched_equals_plain_equals_oracle(k):
    ws = synth.batched_sets(n_sets=12, scale=0.01)
    for w in ws:
        w.params.k = k
    specs, host = make_specs(ws)
    # degenerate sets: no reads, and reads shorter than k
    specs.append(SetSpec(torch.zeros(0, dtype=torch.uint8).cuda(), torch.zeros(0, dtype=torch.uint8).cuda(), 150,
                         10, 10))
    short = np.frombuffer(b"ACGT" * 2000, np.uint8).copy()
    specs.append(SetSpec(torch.from_numpy(short).cuda(), torch.from_numpy(np.full(short.size, 30, np.uint8)).cuda(),
                         20, 1000, 100))
    b = Batch(specs, k, tuning=Tuning(blocks_per_cu=4, tile_bases=4096, list_per_item=4096, slots_per_item=8192))
    b.launch()
    assert all(x == abi.HM_OK for x in b.status())
    batched = [b.table(i) for i in range(len(specs))]
    dig_b = b.digests()
    b.run_plain()
    assert all(x == abi.HM_OK for x in b.status())
    assert b.digests() == dig_b
    for i, r in enumerate(host):
        assert_tables_equal(batched[i], oracle_table(r, k), "set %d" % i)
    assert len(batched[-1]["count"]) == 0 and len(batched[-2]["count"]) == 0


@pytest.mark.parametrize("set_major", [2, 1])  # 1: pass-2 items wait on their own set's pass 1
def test_graph_replays_match_eager(set_major):
    ws = synth.batched_sets(n_sets=8, scale=0.01)
    specs, host = make_specs(ws)
    b = Batch(specs, 31, tuning=Tuning(blocks_per_cu=8, tile_bases=8192, list_per_item=2048, slots_per_item=4096,
                                       set_major=set_major))
    b.launch()
    eager = b.digests()
    b.capture()
    for rep in range(3):
        # the program's own eager work between replays
        b.run_plain()
        assert b.digests() == eager
        b.replay()
        torch.cuda.synchronize()
        assert all(x == abi.HM_OK for x in b.status())
        assert b.digests() == eager, "replay %d" % rep
    assert_tables_equal(b.table(0), oracle_table(host[0], 31), "graph set 0")


def test_output_independent_of_tuning():
    ws = synth.batched_sets(n_sets=6, scale=0.01)
    specs, _ = make_specs(ws)
    ref = None
    for tu in (Tuning(), Tuning(blocks_per_cu=1, tile_bases=1024, list_per_item=256, slots_per_item=2048),
               Tuning(blocks_per_cu=16, table_load=0.6, bloom_bits=6, n_hash=1),
               # lag 0: each set's pass-2 items follow its own pass 1 and wait on its tail (the
               # release/acquire path); phase-major: every pass 1 first
               Tuning(set_major=1, tile_bases=4096, list_per_item=4096), Tuning(set_major=0),
               Tuning(tile_bases=262144), Tuning(tile_bases=16384 + 150)):  # items of many staged runs, ragged
        for in_table in (True, False):
            b = Batch(specs, 31, tuning=tu, bloom_in_table=in_table)
            b.launch()
            st = b.status()
            assert all(x == abi.HM_OK for x in st), (tu, in_table, st)
            d = b.digests()
            ref = ref or d
            assert d == ref
            del b
            torch.cuda.empty_cache()
    # a filter far too small for the table size (sized from the hints, not planned, so the table
    # does not make room for the false positives): false-positive singletons fill the table,
    # which must be reported as a capacity error, never as a wrong table
    b = Batch(specs, 31, tuning=Tuning(table_load=0.9, bloom_bits=1, n_hash=1), plan=False, bloom_in_table=False)
    b.launch()
    st = b.status()
    assert abi.HM_ECAPACITY in st and all(x in (abi.HM_OK, abi.HM_ECAPACITY) for x in st)
    for i, x in enumerate(st):
        if x == abi.HM_OK:
            assert b.digests()[i] == ref[i]


def test_batched_bypass_and_owner_filter():
    ws = synth.batched_sets(n_sets=5, scale=0.01)
    specs, host = make_specs(ws)
    b = Batch(specs, 31, min_depth=1, tuning=Tuning(blocks_per_cu=4, tile_bases=4096))
    b.launch()
    st = b.status()
    assert all(x == abi.HM_OK for x in st), st
    exp = oracle.run(host[1].ascii, host[1].qual, host[1].offsets(), 31, min_depth=1)
    assert_tables_equal(b.table(1), exp, "bypass")
    b = Batch(specs, 31, n_owners=3, owner=2)
    b.launch()
    st = b.status()
    assert all(x == abi.HM_OK for x in st), st
    exp = oracle.run(host[2].ascii, host[2].qual, host[2].offsets(), 31, n_owners=3, owner=2)
    assert_tables_equal(b.table(2), exp, "owner")


def test_autotuner_small():
    from paper_1705_11147_amd import tune
    ws = synth.batched_sets(n_sets=6, scale=0.01)
    specs, _ = make_specs(ws)
    best, rep = tune.autotune(specs, 31, sample=4, reps=1)
    assert isinstance(best, Tuning) and rep["trials"]
