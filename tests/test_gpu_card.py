"""Cardinality pass on the GPU (hm_card_init / hm_cardinality / hm_card_summary, through the C
ABI) against the oracle's (oracle.card).

Everything the pass computes is independent of the order of work, so the bar is exact: the
HyperLogLog registers word by word, the distinct sample's size and kept count, the number of
windows, and the heavy-hitter key set.  The estimate is a double computed from the registers by
the same formula on both sides, summed in a different order: relative tolerance 1e-12."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import random_read_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def gpu_card(ascii, off, k, read_len=None, batches=1, min_depth=2, heavy_min=16, **kw):
    a = torch.from_numpy(np.ascontiguousarray(ascii)).cuda()
    q = torch.full_like(a, 40)
    n_reads = (len(off) - 1)
    P = int(off[-1])  # a bound on the windows
    sk = kmer.CardSketch(k, P, **kw)
    sk.reset()
    cuts = np.linspace(0, n_reads, batches + 1).astype(np.int64)
    for b in range(batches):
        r0, r1 = int(cuts[b]), int(cuts[b + 1])
        if read_len is not None:
            p = kmer.pack_reads(a[r0 * read_len:r1 * read_len], q[r0 * read_len:r1 * read_len], read_len=read_len)
        else:
            o = torch.from_numpy(off[r0:r1 + 1] - off[r0]).cuda()
            p = kmer.pack_reads(a[int(off[r0]):int(off[r1])], q[int(off[r0]):int(off[r1])], read_off=o)
        sk.update(p)
    sk.summarize(min_depth=min_depth, heavy_min=heavy_min)
    return sk, sk.result()


def oracle_card(ascii, off, k, sk, min_depth=2, heavy_min=16, **kw):
    return oracle.card(ascii, off, k, hll_p=sk.hll_p, sample_log2=sk.sample_log2, heavy_log2=sk.heavy_log2,
                       min_depth=min_depth, heavy_min=heavy_min, n_threads=8, **kw)


def assert_card_equal(sk, got, exp, what):
    assert got.status == abi.HM_OK, what
    assert np.array_equal(sk.registers.cpu().numpy().view(np.uint32), exp["registers"]), what + ": registers"
    assert got.positions == exp["positions"], what
    assert got.sampled_distinct == exp["sampled_distinct"], what
    assert got.sampled_kept == exp["sampled_kept"], what
    assert got.n_heavy == exp["n_heavy"], what
    assert np.array_equal(got.heavy_hi, exp["heavy_hi"]) and np.array_equal(got.heavy_lo, exp["heavy_lo"]), what
    assert abs(got.estimate - exp["estimate"]) <= 1e-12 * max(1.0, exp["estimate"]), what


def test_card_tiny_workload():
    """Tiny workload at full size (2e7 windows, k=21): about 2^18 sampled keys and windows."""
    w = synth.tiny()
    r = w.reads()
    sk, got = gpu_card(r.ascii, r.offsets(), 21, read_len=100)
    exp = oracle_card(r.ascii, r.offsets(), 21, sk)
    assert_card_equal(sk, got, exp, "tiny")
    n = len(oracle.run(r.ascii, r.qual, r.offsets(), 21, keep_all=True, n_threads=8)["count"])
    assert abs(got.estimate / n - 1) < 4 * 1.04 / 128


def test_card_mid_shape_two_word_keys_batches():
    """The mid workload's shape at 1/200 (k=51), fed in three batches (the sketch of the union)."""
    w = synth.mid(scale=0.005)
    r = w.reads()
    sk, got = gpu_card(r.ascii, r.offsets(), 51, read_len=150, batches=3)
    exp = oracle_card(r.ascii, r.offsets(), 51, sk)
    assert_card_equal(sk, got, exp, "mid/200")


@pytest.mark.parametrize("k", [1, 5, 21, 31, 33, 63])
def test_card_ragged_reads_all_widths(k):
    """Ragged reads with N and lowercase (the offset path), every key width, small sample rates so
    the samples are not empty."""
    ascii, qual, off = random_read_set(900 + k, 3000, 0, 220, genome_len=30000, n_rate=0.002, lower_rate=0.01)
    sk, got = gpu_card(ascii, off, k, hll_p=12, sample_log2=3, heavy_log2=4, heavy_min=4)
    exp = oracle_card(ascii, off, k, sk, heavy_min=4)
    assert_card_equal(sk, got, exp, "ragged k=%d" % k)


@pytest.mark.parametrize("kw", [dict(forward_only=True), dict(n_owners=4, owner=1), dict(n_owners=4, owner=3)])
def test_card_forward_only_and_owner_filter(kw):
    ascii, qual, off = random_read_set(950, 2000, 100, 150, genome_len=20000)
    k = 32 if kw.get("forward_only") else 31
    sk, got = gpu_card(ascii, off, k, hll_p=10, sample_log2=2, heavy_log2=3, heavy_min=3, **kw)
    exp = oracle_card(ascii, off, k, sk, heavy_min=3, **kw)
    assert_card_equal(sk, got, exp, str(kw))


def test_card_heavy_hitters():
    """Poly-A and (AC)n reads among genome reads: the heavy-hitter set is exact."""
    rng = np.random.default_rng(31)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 100_000)
    n, L = 20_000, 100
    st = rng.integers(0, g.size - L, n)
    reads = [g[s:s + L] for s in st]
    reads += [np.full(L, ord("A"), np.uint8)] * 3000 + [np.frombuffer(b"AC" * (L // 2), np.uint8)] * 2000
    order = rng.permutation(len(reads))
    ascii = np.concatenate([reads[i] for i in order])
    off = np.arange(len(reads) + 1, dtype=np.int64) * L
    sk, got = gpu_card(ascii, off, 21, read_len=L, hll_p=12, sample_log2=4, heavy_log2=6)
    exp = oracle_card(ascii, off, 21, sk)
    assert_card_equal(sk, got, exp, "heavy")
    assert got.n_heavy == 3  # A^21, (AC)^10A, (CA)^10C


def test_card_empty_and_full_table():
    z = np.zeros(0, np.uint8)
    sk, got = gpu_card(z, np.zeros(1, np.int64), 21)
    assert got.estimate == 0.0 and got.positions == 0 and got.status == abi.HM_OK
    # a sample table too small for the sample: reported, and the registers stay exact
    ascii, qual, off = random_read_set(960, 500, 100, 150, genome_len=200000)
    a = torch.from_numpy(ascii).cuda()
    p = kmer.pack_reads(a, torch.full_like(a, 40), read_off=torch.from_numpy(off).cuda())
    sk = kmer.CardSketch(21, 1024, hll_p=10, sample_log2=0, heavy_log2=0)  # sized for 1024 windows
    got = sk.run([p])
    assert got.status == abi.HM_ECAPACITY
    exp = oracle.card(ascii, off, 21, hll_p=10, sample_log2=0, heavy_log2=0)
    assert np.array_equal(sk.registers.cpu().numpy().view(np.uint32), exp["registers"])
    assert got.positions == exp["positions"]


def test_card_sizing_in_analyze():
    """analyze() sized by the cardinality pass gives the oracle's table, on the mid shape."""
    w = synth.mid(scale=0.005)
    r = w.reads()
    got = kmer.analyze(r.ascii, r.qual, 51, read_len=150, fused=True)
    exp = oracle.run(r.ascii, r.qual, r.offsets(), 51, n_threads=8)
    from tests.util import assert_tables_equal
    assert_tables_equal(got, exp, "card-sized mid/200")
    # the plan is not the worst-case bound: the table is at most 1/4 of 2 slots per window
    assert got["capacity"] <= kmer.next_pow2(2 * got["positions"]) // 4


@pytest.mark.parametrize("k,L,fwd", [(1, 40, False), (21, 100, False), (31, 150, False), (33, 150, False),
                                     (51, 150, False), (63, 64, False), (63, 300, False), (32, 100, True),
                                     (2, 30, True)])
def test_card_fixed_length_all_widths(k, L, fwd):
    """Fixed-length reads (the LDS-tiled path that rolls consecutive windows) with N bases, every
    key width, forward-only even k; read lengths with W a multiple of the run and not."""
    rng = np.random.default_rng(k * 1000 + L)
    n = max(50, 400_000 // L)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 50_000)
    st = rng.integers(0, g.size - L, n)
    ascii = np.concatenate([g[s:s + L] for s in st])
    ascii[rng.random(ascii.size) < 0.003] = ord("N")
    e = rng.random(ascii.size) < 0.01
    ascii[e] = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(e.sum()))
    off = np.arange(n + 1, dtype=np.int64) * L
    sk, got = gpu_card(ascii, off, k, read_len=L, hll_p=12, sample_log2=3, heavy_log2=4, heavy_min=4,
                       forward_only=fwd)
    exp = oracle_card(ascii, off, k, sk, heavy_min=4, forward_only=fwd)
    assert_card_equal(sk, got, exp, "fixed k=%d L=%d" % (k, L))


@pytest.mark.parametrize("hll_p", [4, 16])
def test_card_register_count_extremes(hll_p):
    """16 registers (the smallest sketch, alpha_16) and 65536 (64 KB of registers per workgroup)."""
    ascii, qual, off = random_read_set(970 + hll_p, 3000, 100, 150, genome_len=50000)
    sk, got = gpu_card(ascii, off, 31, hll_p=hll_p, sample_log2=2, heavy_log2=3, heavy_min=3)
    exp = oracle_card(ascii, off, 31, sk, heavy_min=3)
    assert_card_equal(sk, got, exp, "p=%d" % hll_p)


def test_card_heavy_list_longer_than_buffer():
    """More heavy hitters than the key buffer holds: the count is complete, the buffer holds a
    subset of the true heavy keys."""
    ascii, qual, off = random_read_set(980, 3000, 100, 150, genome_len=5000)  # deep coverage
    a = torch.from_numpy(ascii).cuda()
    p = kmer.pack_reads(a, torch.full_like(a, 40), read_off=torch.from_numpy(off).cuda())
    sk = kmer.CardSketch(21, int(off[-1]), hll_p=10, sample_log2=0, heavy_log2=0)
    got = sk.run([p], heavy_min=40, heavy_cap=16)
    exp = oracle.card(ascii, off, 21, hll_p=10, sample_log2=0, heavy_log2=0, heavy_min=40)
    assert got.n_heavy == exp["n_heavy"] > 16
    assert len(got.heavy_hi) == 16
    allk = set(zip(exp["heavy_hi"].tolist(), exp["heavy_lo"].tolist()))
    assert set(zip(got.heavy_hi.tolist(), got.heavy_lo.tolist())) <= allk
