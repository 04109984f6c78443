"""Host-side sizing logic (no GPU): the false-positive model of the single-word blocked Bloom
filter (64-bit words of the separate filter, 32-bit words of the filter in the table), and
plan_sizes (table, filter and list sizes from a cardinality pass).

The model is pinned to a Monte Carlo simulation of the filter as the kernels build it (each key's
n_hash bits in one 64-bit word, the word and the bits drawn independently), and to the standard
Bloom formula of section "Parallel k-mer analysis", read with m and n the right way round: at the
loads the filter is built for, a blocked filter is never better than a standard one with the same
bits per key."""
import numpy as np
import pytest

from paper_1705_11147_amd import kmer


def simulate_fp(bits_per_key: float, n_hash: int, n_words: int = 1 << 13, n_test: int = 200_000, seed: int = 0,
                word_bits: int = 64):
    rng = np.random.default_rng(seed)
    n_keys = int(n_words * word_bits / bits_per_key)
    words = np.zeros(n_words, np.uint64)
    w = rng.integers(0, n_words, n_keys)
    mask = np.zeros(n_keys, np.uint64)
    for _ in range(n_hash):
        mask |= np.left_shift(np.uint64(1), rng.integers(0, word_bits, n_keys).astype(np.uint64))
    np.bitwise_or.at(words, w, mask)
    tw = rng.integers(0, n_words, n_test)
    tm = np.zeros(n_test, np.uint64)
    for _ in range(n_hash):
        tm |= np.left_shift(np.uint64(1), rng.integers(0, word_bits, n_test).astype(np.uint64))
    return float(np.mean((words[tw] & tm) == tm)), n_test


@pytest.mark.parametrize("word_bits", [64, 32])
@pytest.mark.parametrize("bits_per_key", [4.0, 8.0, 12.0, 18.0])
@pytest.mark.parametrize("n_hash", [1, 2, 4, 6])
def test_blocked_bloom_model_matches_simulation(bits_per_key, n_hash, word_bits):
    p, n = simulate_fp(bits_per_key, n_hash, seed=int(bits_per_key * 10 + n_hash + word_bits), word_bits=word_bits)
    model = kmer.bloom_fp_rate(bits_per_key, n_hash, word_bits=word_bits)
    sigma = max((model * (1 - model) / n) ** 0.5, 1.0 / n)
    assert abs(p - model) <= 5 * sigma + 0.02 * model, (p, model)


@pytest.mark.parametrize("word_bits", [64, 32])
@pytest.mark.parametrize("bits_per_key", [6.0, 12.0, 24.0])
@pytest.mark.parametrize("n_hash", [1, 3, 4, 8])
def test_blocked_bloom_never_beats_the_standard_formula(bits_per_key, n_hash, word_bits):
    """In the sizes the filter is built for (6 to 24 bits per key, a few keys per word) the
    per-word false-positive rate is convex in the word's load, so the uneven load of the blocks
    can only raise the rate above the standard formula's (far beyond, at tens of keys per word, it
    turns concave and the inequality no longer holds).  Smaller words spread the load less
    evenly: at the same bits per key a 32-bit-word filter errs at least as often as a 64-bit one."""
    standard = (1.0 - np.exp(-n_hash / bits_per_key)) ** n_hash  # FP = (1 - e^{-h n / m})^h, m / n = bits per key
    blocked = kmer.bloom_fp_rate(bits_per_key, n_hash, word_bits=word_bits)
    assert blocked >= standard * (1 - 1e-9)
    if word_bits == 32:
        assert blocked >= kmer.bloom_fp_rate(bits_per_key, n_hash) * (1 - 1e-9)
    # with one bit per key the words' load does not matter beyond the bit collisions in a word
    if n_hash == 1:
        assert blocked == pytest.approx(1.0 - np.exp(-1.0 / bits_per_key), rel=0.02)


def test_blocked_bloom_model_limits():
    assert kmer.bloom_fp_rate(1e9, 4) < 1e-12       # an empty filter
    assert kmer.bloom_fp_rate(1e-3, 4) > 0.999      # a saturated one
    rates = [kmer.bloom_fp_rate(b, 4) for b in (4, 8, 12, 16, 24)]
    assert all(x > y for x, y in zip(rates, rates[1:]))  # more bits per key, fewer false positives


def card(estimate=4.0e8, kept=12000, sample_log2=13, hll_p=14):
    return kmer.CardResult(estimate=estimate, sampled_distinct=50000, sampled_kept=kept, n_heavy=0,
                           positions=2_000_000_000, hll_p=hll_p, sample_log2=sample_log2, heavy_log2=13,
                           heavy_hi=np.zeros(0, np.uint64), heavy_lo=np.zeros(0, np.uint64), status=0)


@pytest.mark.parametrize("in_table", [False, True])
def test_plan_sizes(monkeypatch, in_table):
    monkeypatch.setattr(kmer, "list_slack", lambda pass1_launches=1, device=None: 1000 * pass1_launches)
    c = card()
    cap, words, lcap = kmer.plan_sizes(c, n_hash=4, bloom_bits=12.0, table_load=0.5, bloom_in_table=in_table)
    assert cap & (cap - 1) == 0 and words & (words - 1) == 0
    assert words * 64 >= c.distinct_hi() * 12.0 and words * 64 < 2 * c.distinct_hi() * 12.0 + 128
    assert cap * 0.5 >= c.kept_hi()          # the kept k-mers fit at the design load
    assert lcap >= c.distinct_hi() + 1000    # one first occurrence per distinct k-mer, plus the slack
    if in_table:  # 32 filter bits per slot: the table holds at least the filter's bits
        assert cap * 32 >= words * 64
    else:  # a bigger filter lets fewer singletons into the table
        cap2, _, _ = kmer.plan_sizes(c, n_hash=4, bloom_bits=2.0, table_load=0.5, bloom_in_table=False)
        assert cap2 >= cap
    # at the design's 12 bits per key the filter's false positives stay a small part of the table
    fp = kmer.bloom_fp_rate(cap * 32 / c.distinct_hi() if in_table else words * 64 / c.distinct_hi(), 4,
                            word_bits=32 if in_table else 64)
    assert fp * (c.distinct_hi() - c.kept_hi()) < 0.05 * cap
    # the kept bound: Poisson margin on the sample, never above the distinct bound
    assert c.kept_hi() == pytest.approx((12000 + 4 * 12000 ** 0.5 + 4) * 2 ** 13)
    assert card(estimate=1000.0, kept=12000).kept_hi() == pytest.approx(card(estimate=1000.0).distinct_hi())
