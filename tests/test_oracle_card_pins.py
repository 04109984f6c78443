"""Pins of the oracle's cardinality pass (section "Parallel k-mer analysis": the HyperLogLog
estimate of distinct k-mers that sizes the Bloom filter, merged across workers by keeping the
larger register; heavy hitters found in the same pass).

References, none of them the oracle itself: a Python brute force over string slices
(tests/brute.card), the exact distinct and kept counts of the oracle's own table run (pinned in
test_oracle_pins.py), the HyperLogLog error bound 1.04/sqrt(m), and the merge identity."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests import brute
from tests.util import pack_reads

BASES = "ACGT"
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def card_reads(seqs, k, **kw):
    a, _, off = pack_reads([(s, [40] * len(s)) for s in seqs])
    return oracle.card(a, off, k, **kw)


def key_of(hi, lo):
    return (int(hi) << 64) | int(lo)


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seqs=st.lists(st.text(alphabet="ACGTNacgt", min_size=0, max_size=60), min_size=0, max_size=10),
       k=st.sampled_from([1, 3, 5, 7, 33]), hll_p=st.integers(4, 8), sample_log2=st.integers(0, 3),
       heavy_log2=st.integers(0, 3), min_depth=st.integers(1, 3), heavy_min=st.integers(1, 3),
       n_owners=st.sampled_from([1, 3]), fwd=st.booleans(), threads=st.sampled_from([1, 3]))
def test_card_equals_brute_force(seqs, k, hll_p, sample_log2, heavy_log2, min_depth, heavy_min, n_owners, fwd,
                                 threads):
    seqs = seqs + seqs[: len(seqs) // 2]  # repeats, so that counts reach the thresholds
    for own in range(n_owners):
        exp = brute.card(seqs, k, hll_p, sample_log2, heavy_log2, min_depth, heavy_min, forward_only=fwd,
                         n_owners=n_owners, own=own)
        got = card_reads(seqs, k, hll_p=hll_p, sample_log2=sample_log2, heavy_log2=heavy_log2, min_depth=min_depth,
                         heavy_min=heavy_min, forward_only=fwd, n_owners=n_owners, owner=own, n_threads=threads)
        assert list(got["registers"]) == exp["registers"]
        assert got["sampled_distinct"] == exp["sampled_distinct"]
        assert got["sampled_kept"] == exp["sampled_kept"]
        assert got["positions"] == exp["positions"]
        assert [key_of(h, l) for h, l in zip(got["heavy_hi"], got["heavy_lo"])] == exp["heavy"]


def random_distinct_reads(rng, n_reads, L):
    """Independent random reads: with k >= 21 every window is a distinct k-mer with overwhelming
    probability, and the oracle's exact table gives the true number anyway."""
    a = rng.choice(np.frombuffer(b"ACGT", np.uint8), n_reads * L)
    return a, np.arange(n_reads + 1, dtype=np.int64) * L


@pytest.mark.parametrize("hll_p", [10, 14])
@pytest.mark.parametrize("n_reads", [3, 40, 400, 4000, 40000])
def test_estimate_within_hll_error_bound(hll_p, n_reads):
    """|E - n| <= 4 * 1.04 / sqrt(m) * n over cardinalities from far below m (linear counting) to
    far above it; n is the exact number of distinct keys from the oracle's table."""
    rng = np.random.default_rng(1000 * hll_p + n_reads)
    a, off = random_distinct_reads(rng, n_reads, 100)
    exact = len(oracle.run(a, np.full(a.size, 40, np.uint8), off, 21, keep_all=True, n_threads=4)["count"])
    got = oracle.card(a, off, 21, hll_p=hll_p, n_threads=4)
    bound = 4 * 1.04 / math.sqrt(1 << hll_p)
    assert abs(got["estimate"] - exact) <= bound * exact + 1, (got["estimate"], exact)


def test_estimate_bias_over_many_sketches():
    """Averaged over 32 independent inputs the relative error shrinks as 1/sqrt(32): a constant
    bias (a wrong alpha_m, an off-by-one rank) shows up here even when one sketch hides it."""
    rng = np.random.default_rng(77)
    errs = []
    for _ in range(32):
        a, off = random_distinct_reads(rng, 2000, 100)
        exact = len(oracle.run(a, np.full(a.size, 40, np.uint8), off, 21, keep_all=True)["count"])
        errs.append(oracle.card(a, off, 21, hll_p=10)["estimate"] / exact - 1)
    assert abs(np.mean(errs)) <= 4 * 1.04 / math.sqrt(1 << 10) / math.sqrt(32)
    assert 0.5 * 1.04 / 32 <= np.std(errs) <= 2 * 1.04 / 32  # sqrt(m) = 32 at p = 10


def test_empty_sketch_estimates_zero():
    a, off = random_distinct_reads(np.random.default_rng(0), 0, 100)
    got = oracle.card(a, off, 21)
    assert got["estimate"] == 0.0 and not got["registers"].any() and got["positions"] == 0


def test_merge_is_register_maximum():
    """The paper's merge of sketches: the sketch of the union of two read sets is the
    register-wise maximum of their sketches."""
    rng = np.random.default_rng(3)
    a1, off1 = random_distinct_reads(rng, 500, 120)
    a2, off2 = random_distinct_reads(rng, 700, 90)
    a = np.concatenate([a1, a2])
    off = np.concatenate([off1, off2[1:] + off1[-1]])
    r1 = oracle.card(a1, off1, 31)["registers"]
    r2 = oracle.card(a2, off2, 31)["registers"]
    ru = oracle.card(a, off, 31, n_threads=3)["registers"]
    assert np.array_equal(ru, np.maximum(r1, r2))


def sample_pred(hi, lo, s):
    h = brute.fmix64(brute.fmix64(int(hi) ^ 0xB7E151628AED2A6A) ^ int(lo))
    return h % (1 << s) == 0


def test_sample_counts_match_exact_table():
    """The distinct sample is exactly the keys of the exact table that satisfy the sampling
    predicate (computed here in Python), and its kept count those with count >= min_depth; scaled
    by 2^s, the kept count estimates the table's within 5 standard deviations."""
    rng = np.random.default_rng(11)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 200_000)
    n, L = 40_000, 100
    st_ = rng.integers(0, g.size - L, n)
    a = np.concatenate([g[s:s + L] for s in st_])
    err = rng.random(a.size) < 0.01
    a[err] = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(err.sum()))
    off = np.arange(n + 1, dtype=np.int64) * L
    q = np.full(a.size, 40, np.uint8)
    s = 6
    allk = oracle.run(a, q, off, 21, keep_all=True, n_threads=4)
    kept = oracle.run(a, q, off, 21, min_depth=2, n_threads=4)
    got = oracle.card(a, off, 21, sample_log2=s, min_depth=2, n_threads=4)
    in_all = sum(sample_pred(h, l, s) for h, l in zip(allk["key_hi"], allk["key_lo"]))
    in_kept = sum(sample_pred(h, l, s) for h, l in zip(kept["key_hi"], kept["key_lo"]))
    assert got["sampled_distinct"] == in_all
    assert got["sampled_kept"] == in_kept
    n_kept = len(kept["count"])
    sigma = math.sqrt(n_kept * (1 << s))
    assert abs(got["sampled_kept"] * (1 << s) - n_kept) <= 5 * sigma


def test_heavy_hitters_found_and_exact():
    """Reads of a poly-A run and of an (AC)n microsatellite among random reads: their k-mers are
    the heavy hitters, and the oracle's list equals the brute force's."""
    rng = np.random.default_rng(5)
    g = "".join(rng.choice(list(BASES), 50_000))
    seqs = []
    for _ in range(1500):
        s = int(rng.integers(0, len(g) - 100))
        seqs.append(g[s:s + 100])
    seqs += ["A" * 100] * 300 + ["AC" * 50] * 200
    rng.shuffle(seqs)
    k = 21
    exp = brute.card(seqs, k, 10, 4, 6, 2, 16)
    got = card_reads(seqs, k, hll_p=10, sample_log2=4, heavy_log2=6, min_depth=2, heavy_min=16, n_threads=2)
    heavy = [key_of(h, l) for h, l in zip(got["heavy_hi"], got["heavy_lo"])]
    assert heavy == exp["heavy"]
    polya = brute.enc("A" * k)
    ac = min(brute.enc(("AC" * k)[:k]), brute.enc(brute.revcomp(("AC" * k)[:k])))
    ca = min(brute.enc(("CA" * k)[:k]), brute.enc(brute.revcomp(("CA" * k)[:k])))
    assert set(heavy) == {polya, ac, ca}
