"""The binned path (hm_bin_kmers, hm_count_bins; spilled bins through the global-table path and
hm_export_merge) against the CPU oracle, record by record.

Integer output: the bar is bit-exact equality of the sorted tables (keys, counts, both tally
arrays, both class bytes) and of the order-free digest."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, random_read_set, table_digest

pytestmark = pytest.mark.gpu

OKW = ("qcut", "min_depth", "ext_min", "n_owners", "owner", "qual_offset", "forward_only")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def fixed_reads(seed, n_reads, L, genome_len, err=0.01, n_rate=0.0, lower_rate=0.0):
    ascii, qual, _ = random_read_set(seed, n_reads, L, L, genome_len, err, n_rate, lower_rate)
    return ascii, qual


def run_both(ascii, qual, L, k, bin_bits=None, **kw):
    n = ascii.size // L if L else 0
    off = np.arange(n + 1, dtype=np.int64) * L
    got = kmer.analyze(ascii, qual, k, read_len=L, binned=True, bin_bits=bin_bits, **kw)
    exp = oracle.run(ascii, qual, off, k, n_threads=8, sort_count=True, **{x: kw[x] for x in OKW if x in kw})
    return got, exp


def valid_windows(ascii, L, k):
    """Windows of the fixed-length reads that hold only A/C/G/T (either case)."""
    if ascii.size == 0 or L < k:
        return 0
    bad = ~np.isin(ascii | 0x20, np.frombuffer(b"acgt", np.uint8)).reshape(-1, L)
    c = np.concatenate([np.zeros((bad.shape[0], 1), np.int64), np.cumsum(bad, axis=1)], axis=1)
    return int(((c[:, k:] - c[:, :-k]) == 0).sum())


def check(got, exp, what, ascii=None, L=None, k=None):
    assert_tables_equal(got, exp, what)
    assert got["digest"] == table_digest(exp), what
    if ascii is not None:  # every valid window went into a bin once
        assert got["bin_stats"]["records"] == valid_windows(ascii, L, k), what


@pytest.mark.parametrize("k,L,n_reads,G,err,n_rate,lower", [
    (21, 100, 20000, 50000, 0.01, 0.0, 0.0),
    (51, 150, 10000, 100000, 0.005, 0.0, 0.0),
    (31, 150, 10000, 60000, 0.01, 0.0, 0.0),
    (61, 150, 5000, 40000, 0.01, 0.0, 0.0),   # the largest k of the binned path
    (33, 100, 4000, 20000, 0.01, 0.0, 0.0),   # keys just past one 64-bit word
    (25, 120, 5000, 30000, 0.01, 0.01, 0.1),  # N bases and lowercase
    (3, 40, 2000, 500, 0.02, 0.0, 0.0),       # 32 canonical 3-mers, huge counts
    (1, 50, 500, 1000, 0.0, 0.0, 0.0),        # two canonical 1-mers
])
def test_binned_matches_oracle(k, L, n_reads, G, err, n_rate, lower):
    print("binned k=%d L=%d reads=%d G=%d" % (k, L, n_reads, G), flush=True)
    ascii, qual = fixed_reads(1000 + k, n_reads, L, G, err, n_rate, lower)
    got, exp = run_both(ascii, qual, L, k)
    check(got, exp, "k=%d" % k, ascii, L, k)


@pytest.mark.parametrize("kw", [dict(forward_only=True), dict(min_depth=3, ext_min=1), dict(min_depth=2, ext_min=3),
                                dict(n_owners=4, owner=1), dict(qcut=30), dict(seed=12345)])
def test_binned_params(kw):
    print("binned params %r" % kw, flush=True)
    ascii, qual = fixed_reads(77, 8000, 100, 40000, 0.01)
    got, exp = run_both(ascii, qual, 100, 21, **kw)
    check(got, exp, repr(kw), None if "n_owners" in kw else ascii, 100, 21)


def test_binned_uu_only():
    ascii, qual = fixed_reads(78, 8000, 100, 40000, 0.01)
    got, exp = run_both(ascii, qual, 100, 21, export_flags=abi.HM_EXPORT_UU_ONLY)
    uu = (exp["cls_l"] < 4) & (exp["cls_r"] < 4)
    exp = {f: (v[uu] if isinstance(v, np.ndarray) and len(v) == len(uu) else v) for f, v in exp.items()}
    assert_tables_equal(got, exp, "UU only")
    assert got["digest"] == table_digest(exp)


def test_every_bin_spills():
    """One bin holding every record, with far more repeated k-mers than its local table takes:
    the bin goes whole to the spill stream and the global-table path counts it."""
    ascii, qual = fixed_reads(79, 6000, 100, 20000, 0.01)
    got, exp = run_both(ascii, qual, 100, 21, bin_bits=(0, 0))
    check(got, exp, "one bin", ascii, 100, 21)
    assert got["bin_stats"]["spilled_bins"] == 1 and got["spilled"] == valid_windows(ascii, 100, 21)


def test_some_bins_spill():
    """Eight bins for about 2900 repeated k-mers (320 to 390 a bin, around the spill limit of 384): some
    bins are counted locally, the others through the global path, and the merged export is exact."""
    ascii, qual = fixed_reads(80, 4000, 100, 2600, 0.002)
    got, exp = run_both(ascii, qual, 100, 21, bin_bits=(1, 2))
    check(got, exp, "mixed")
    st = got["bin_stats"]
    print("spilled bins %d of 8, %d records" % (st["spilled_bins"], st["spilled"]), flush=True)
    assert 0 < st["spilled_bins"] < 8


def test_deferred_list_spills():
    """A bin whose distinct k-mers pass its deferred list (2048): error-rich reads, one bin."""
    ascii, qual = fixed_reads(81, 800, 100, 200000, 0.05)
    got, exp = run_both(ascii, qual, 100, 21, bin_bits=(0, 0))
    check(got, exp, "deferred overflow")
    assert got["bin_stats"]["spilled_bins"] == 1


@pytest.mark.parametrize("bin_bits", [None, (0, 1)])
def test_bypass(bin_bits):
    """min_depth = 1: no Bloom filter, every k-mer inserted (with (0, 1) both bins spill)."""
    ascii, qual = fixed_reads(82, 3000, 100, 20000, 0.01)
    got, exp = run_both(ascii, qual, 100, 21, bin_bits=bin_bits, min_depth=1)
    check(got, exp, "bypass %r" % (bin_bits,))


def test_heavy_hitter_bin():
    """A k-mer in 20% of the windows: its bin takes a third of all records and one slot's counters
    take every one of its occurrences."""
    ascii, qual = fixed_reads(83, 10000, 100, 40000, 0.01)
    ascii = ascii.reshape(10000, 100)
    ascii[::5] = ord("A")  # 2000 poly-A reads: 80 windows each of the key A...A
    got, exp = run_both(ascii.reshape(-1).copy(), qual, 100, 21)
    check(got, exp, "heavy")
    assert int(exp["count"].max()) >= 160000


@pytest.mark.parametrize("n_reads,L,k", [(0, 100, 21), (50, 20, 21), (1, 21, 21)])
def test_degenerate(n_reads, L, k):
    """No reads, reads shorter than k, one read of exactly k bases."""
    ascii, qual = fixed_reads(84, n_reads, L, 1000, 0.0) if n_reads else (np.zeros(0, np.uint8), np.zeros(0, np.uint8))
    got, exp = run_both(ascii, qual, L, k, min_depth=1)
    check(got, exp, "degenerate", ascii, L, k)


def test_binned_equals_table_path_mid_scale():
    """The mid workload at 1/100 scale (2*10^7 windows, about 2^14 bins): the binned export equals
    the oracle's table and the global-table path's, record by record."""
    w = synth.mid(scale=0.01)
    r = w.reads()
    p = w.params
    got, exp = run_both(r.ascii, r.qual, r.read_len, p.k, qcut=p.qcut, min_depth=p.min_depth)
    check(got, exp, "mid 0.01")
    tab = kmer.analyze(r.ascii, r.qual, p.k, read_len=r.read_len, qcut=p.qcut, min_depth=p.min_depth)
    assert_tables_equal(got, tab, "binned vs table path")
    assert got["spilled"] == 0


def _bins_by_bin(bc):
    """(bin, key_lo, key_hi | ext << 58) of every record that is not padding, sorted.  The order
    inside a bin, and so the padding, follow the partition's schedule; which records a bin holds
    does not."""
    start = bc.bin_start.cpu().numpy()
    n = int(start[-1])
    recs = bc.recs[: 2 * n].cpu().numpy().view(np.uint64).reshape(-1, 2)
    bin_id = np.repeat(np.arange(len(start) - 1, dtype=np.uint64), np.diff(start))
    keep = (recs[:, 1] >> np.uint64(58)) != 63  # holes: extension field 63
    t = np.stack([bin_id[keep], recs[keep, 0], recs[keep, 1]], axis=1)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


@pytest.mark.parametrize("k,L,kw", [(21, 100, {}), (51, 150, dict(n_owners=4, owner=1)), (31, 150, dict(forward_only=True))])
def test_histogram_counted_by_the_cardinality_pass(k, L, kw):
    """hm_cardinality_bins + hm_bin_kmers(HM_BINS_COUNTED) against hm_cardinality + hm_bin_kmers: every
    bin holds the same records, the HyperLogLog registers and the sample summary are the same, and
    the counted export equals the oracle's."""
    print("fused histogram k=%d L=%d %r" % (k, L, kw), flush=True)
    ascii, qual = fixed_reads(90 + k, 12000, L, 60000, 0.01)
    dev = torch.device("cuda")
    packed = kmer.pack_reads(torch.from_numpy(ascii).to(dev), torch.from_numpy(qual).to(dev), read_len=L)
    P = packed.positions(k)
    n_owners, owner = kw.get("n_owners", 1), kw.get("owner", 0)
    fwd = kw.get("forward_only", False)
    flags = abi.HM_FORWARD_ONLY if fwd else 0
    got = []
    for fused in (False, True):
        sk = kmer.CardSketch(k, P, n_owners=n_owners, owner=owner, forward_only=fwd, device=dev)
        bc = kmer.BinnedCounter(k, P, 3, 6, n_owners=n_owners, owner=owner, flags=flags, device=dev)
        sk.reset()
        sk.update(packed, bins=bc if fused else None)
        bc.bin(packed, counted=fused)
        sk.summarize(min_depth=2)
        fetched = sk.fetch()
        torch.cuda.synchronize()
        res = sk.decode(fetched)
        out = kmer.Records(max(1024, P), device=dev)
        bc.count(out)
        assert bc.finish(out) == 0
        abi.check(bc.status(), "binned")
        tab = out.to_numpy(sort=True)
        got.append((_bins_by_bin(bc), sk.registers.cpu().numpy().copy(), res, tab, bc.stats()))
    b0, reg0, c0, t0, st0 = got[0]
    b1, reg1, c1, t1, st1 = got[1]
    assert np.array_equal(b0, b1)
    assert np.array_equal(reg0, reg1)
    assert (c0.estimate, c0.sampled_distinct, c0.sampled_kept, c0.positions) == \
        (c1.estimate, c1.sampled_distinct, c1.sampled_kept, c1.positions)
    # keys inserted and occurrences deferred follow the order inside a bin (a Bloom false positive
    # lets a k-mer in early); the rest does not
    fixed = ("records", "spilled_bins", "spilled", "kept")
    assert {x: st0[x] for x in fixed} == {x: st1[x] for x in fixed}
    off = np.arange(ascii.size // L + 1, dtype=np.int64) * L
    exp = oracle.run(ascii, qual, off, k, n_threads=8, sort_count=True, **kw)
    assert_tables_equal(t1, exp, "fused histogram")
    if n_owners == 1:
        assert st1["records"] == valid_windows(ascii, L, k)


def _stream_run(ascii, qual, L, k, batches, n_owners, owner, bin_bits=None):
    """The owner's occurrences written to a stream by the cardinality pass (one launch a batch, so
    the stream has holes), partitioned from the stream and counted in bins."""
    dev = torch.device("cuda")
    n = ascii.size // L
    cuts = np.linspace(0, n, batches + 1).astype(np.int64)
    packs = [kmer.pack_reads(torch.from_numpy(ascii[a * L:b * L].copy()).to(dev),
                             torch.from_numpy(qual[a * L:b * L].copy()).to(dev), read_len=L)
             for a, b in zip(cuts[:-1], cuts[1:])]
    P = n * (L - k + 1)
    sk = kmer.CardSketch(k, P, n_owners=n_owners, owner=owner, device=dev)
    occ = kmer.OccStream.for_windows(P, n_owners, batches, device=dev)
    card = sk.run(packs, min_depth=2, occ=occ)
    assert not occ.overflowed()
    g, b = bin_bits if bin_bits is not None else kmer.plan_bins(card.distinct_hi(), card.kept_hi(), False)
    bc = kmer.BinnedCounter(k, occ.capacity, g, b, n_owners=n_owners, owner=owner, device=dev)
    out = kmer.Records(max(1024, P // max(n_owners, 1)), device=dev)
    bc.bin_occ(occ)
    bc.count(out)
    spilled = bc.finish(out)
    abi.check(bc.status(), "binned from a stream")
    res = out.to_numpy(sort=True)
    res["digest"] = out.digest_words()
    return res, spilled, bc.stats(), card


@pytest.mark.parametrize("k,L,batches,n_owners,owner", [(21, 100, 2, 4, 1), (51, 150, 3, 3, 2), (31, 150, 1, 1, 0)])
def test_binned_from_occurrence_stream(k, L, batches, n_owners, owner):
    """hm_cardinality_occ writes one owner's occurrences, hm_bin_occ partitions the stream and
    hm_count_bins counts it: the oracle's table of that owner, record by record."""
    print("stream k=%d L=%d batches=%d owner %d of %d" % (k, L, batches, owner, n_owners), flush=True)
    ascii, qual = fixed_reads(95 + k, 12000, L, 60000, 0.01)
    got, spilled, st, card = _stream_run(ascii, qual, L, k, batches, n_owners, owner)
    off = np.arange(ascii.size // L + 1, dtype=np.int64) * L
    exp = oracle.run(ascii, qual, off, k, n_threads=8, sort_count=True, n_owners=n_owners, owner=owner)
    assert_tables_equal(got, exp, "stream k=%d" % k)
    assert got["digest"] == table_digest(exp)
    assert st["records"] == card.positions  # every owned occurrence, none of the holes


def test_binned_from_stream_spills():
    """One bin for the whole stream: it spills and the table path counts it from the spill stream."""
    ascii, qual = fixed_reads(97, 4000, 100, 20000, 0.01)
    got, spilled, st, card = _stream_run(ascii, qual, 100, 21, 2, 2, 1, bin_bits=(0, 0))
    off = np.arange(ascii.size // 100 + 1, dtype=np.int64) * 100
    exp = oracle.run(ascii, qual, off, 21, n_threads=8, sort_count=True, n_owners=2, owner=1)
    assert_tables_equal(got, exp, "stream spill")
    # the spill stream holds the bin's range, padding included; its records are the owned occurrences
    assert st["spilled_bins"] == 1 and st["spilled"] == card.positions and spilled >= card.positions


@pytest.mark.parametrize("n_owners,owner", [(3, 1), (1, 0)])
def test_analyze_binned_from_stream(n_owners, owner):
    """kmer.analyze(binned=True, occ_stream=True): the cardinality pass writes the owned occurrences
    and the bins are filled from that stream; the table equals the oracle's for that owner."""
    ascii, qual = fixed_reads(98, 8000, 120, 40000, 0.01)
    got, exp = run_both(ascii, qual, 120, 31, n_owners=n_owners, owner=owner, occ_stream=True)
    check(got, exp, "analyze stream %d of %d" % (owner, n_owners))
