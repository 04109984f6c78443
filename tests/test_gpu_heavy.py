"""Heavy hitters counted in workgroup-local memory (hm_table_t.heavy) against the oracle.

Whatever keys the list holds, every occurrence is still counted exactly once, so the bar is the
same bit-exact table as without the list."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, random_read_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def with_satellites(seed, n_reads=20_000, L=100, genome_len=100_000, poly=3000, micro=2000):
    rng = np.random.default_rng(seed)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), genome_len)
    st = rng.integers(0, g.size - L, n_reads)
    reads = [g[s:s + L].copy() for s in st]
    reads += [np.full(L, ord("A"), np.uint8) for _ in range(poly)]
    reads += [np.frombuffer(b"CA" * (L // 2), np.uint8).copy() for _ in range(micro)]
    reads = [reads[i] for i in rng.permutation(len(reads))]
    for r in reads:  # sequencing errors, so the satellites have error neighbours too
        e = rng.random(L) < 0.005
        r[e] = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(e.sum()))
    ascii = np.concatenate(reads)
    qual = rng.integers(2, 42, ascii.size).astype(np.uint8)
    return ascii, qual, np.arange(len(reads) + 1, dtype=np.int64) * L


def run_counter(ascii, qual, off, k, heavy, read_len=None, batches=((0, None),), flags=0, min_depth=2,
                export_flags=0, n_owners=1, owner=0):
    a = torch.from_numpy(ascii).cuda()
    q = torch.from_numpy(qual).cuda()
    P = int(off[-1])
    kc = kmer.KmerCounter(k, kmer.next_pow2(2 * P), kmer.next_pow2(P // 4 + 64), P + kmer.list_slack(4),
                          min_depth=min_depth, flags=flags, heavy=heavy, n_owners=n_owners, owner=owner)
    kc.reset()
    n_heavy = kc.table.n_heavy
    for r0, r1 in batches:
        r1 = len(off) - 1 if r1 is None else r1
        if read_len:
            p = kmer.pack_reads(a[r0 * read_len:r1 * read_len], q[r0 * read_len:r1 * read_len], read_len=read_len)
        else:
            o = torch.from_numpy(off[r0:r1 + 1] - off[r0]).cuda()
            p = kmer.pack_reads(a[int(off[r0]):int(off[r1])], q[int(off[r0]):int(off[r1])], read_off=o)
        kc.insert(p)
        kc.table.n_heavy = 0  # later batches (if any) count heavy keys through the table
    kc.table.n_heavy = n_heavy
    kc.count()
    out = kmer.Records(kc.capacity)
    kc.export(out, export_flags | abi.HM_EXPORT_CLASSIFY)
    abi.check(kc.status(), "heavy test")
    return out.to_numpy(), kc.stats()


def keys_of(t, idx):
    return np.stack([t["key_hi"][idx], t["key_lo"][idx]], axis=1)


def test_heavy_workload_shape_exact():
    """mid-heavy at 1/200 through analyze(): the cardinality pass finds the satellite k-mers,
    pass 1 counts them locally, and the table equals the oracle's."""
    w = synth.mid_heavy(scale=0.005)
    r = w.reads()
    got = kmer.analyze(r.ascii, r.qual, 51, read_len=150, fused=True)
    exp = oracle.run(r.ascii, r.qual, r.offsets(), 51, n_threads=8)
    assert_tables_equal(got, exp, "mid-heavy/200")
    assert got["n_heavy"] > 0 and got["stats"]["heavy_local"] > 0


@pytest.mark.parametrize("k", [21, 51])
def test_arbitrary_heavy_lists_are_exact(k):
    """Top keys, keys that never occur, duplicated keys: counts unchanged; absent keys never
    appear in the output, also with HM_EXPORT_ALL."""
    ascii, qual, off = with_satellites(40 + k)
    exp = oracle.run(ascii, qual, off, k, n_threads=8)
    top = np.argsort(exp["count"])[::-1][:40]
    absent = np.array([[0, 12345], [1 if k > 32 else 0, 999]], np.uint64)
    heavy = np.concatenate([keys_of(exp, top), absent, keys_of(exp, top[:5])])
    got, st = run_counter(ascii, qual, off, k, heavy, read_len=100)
    assert_tables_equal(got, exp, "k=%d" % k)
    assert st["heavy_local"] > 0.1 * st["occurrences"]
    allk, _ = run_counter(ascii, qual, off, k, heavy, read_len=100, export_flags=abi.HM_EXPORT_ALL)
    present = set(zip(allk["key_hi"].tolist(), allk["key_lo"].tolist()))
    assert not any((int(h), int(l)) in present for h, l in absent)


def test_full_heavy_list_var_path_and_bypass():
    ascii, qual, off = random_read_set(77, 3000, 0, 220, genome_len=30000, n_rate=0.002)
    exp = oracle.run(ascii, qual, off, 31, n_threads=8)
    heavy = keys_of(exp, np.argsort(exp["count"])[::-1][:abi.HM_MAX_HEAVY])
    assert len(heavy) == abi.HM_MAX_HEAVY
    got, _ = run_counter(ascii, qual, off, 31, heavy)
    assert_tables_equal(got, exp, "256 keys, offsets path")
    got, _ = run_counter(ascii, qual, off, 31, heavy, flags=abi.HM_BLOOM_BYPASS)
    assert_tables_equal(got, exp, "bypass")
    expall = oracle.run(ascii, qual, off, 31, min_depth=1, n_threads=8)
    got, _ = run_counter(ascii, qual, off, 31, heavy, min_depth=1)
    assert_tables_equal(got, expall, "min_depth 1")


def test_heavy_then_plain_batches_and_owner_filter():
    """Batch 1 with the heavy list, batch 2 without it, one table; and a list holding keys of
    other owners under the owner filter."""
    ascii, qual, off = with_satellites(9)
    n = len(off) - 1
    exp = oracle.run(ascii, qual, off, 21, n_threads=8)
    heavy = keys_of(exp, np.argsort(exp["count"])[::-1][:20])
    got, _ = run_counter(ascii, qual, off, 21, heavy, read_len=100, batches=((0, n // 2), (n // 2, n)))
    assert_tables_equal(got, exp, "heavy then plain")
    expo = oracle.run(ascii, qual, off, 21, n_owners=4, owner=2, n_threads=8)
    got, _ = run_counter(ascii, qual, off, 21, heavy, read_len=100, n_owners=4, owner=2)
    assert_tables_equal(got, expo, "owner 2 of 4")
