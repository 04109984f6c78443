"""The owned-occurrence stream (hm_cardinality_occ + hm_bloom_insert_occ)
against the CPU oracle, record by record (integer output: tolerance 0).

The cardinality pass writes every owned occurrence with its extensions, and
pass 1 reads that stream instead of scanning the reads again; the table must
be the one the plain definition gives for the same owner filter."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, random_read_set, table_digest

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def both(ascii, qual, off, k, read_len=None, **kw):
    okw = {x: kw[x] for x in ("qcut", "min_depth", "ext_min", "n_owners", "owner", "forward_only") if x in kw}
    got = kmer.analyze(ascii, qual, k, read_len=read_len, read_off=None if read_len else off, occ_stream=True, **kw)
    exp = oracle.run(ascii, qual, off, k, n_threads=4, **okw)
    return got, exp


def fixed_reads(seed, k, L, n, genome_len=20000, err=0.01):
    rng = np.random.default_rng(seed)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), genome_len)
    starts = rng.integers(0, g.size - L + 1, n)
    ascii = np.concatenate([g[s:s + L] for s in starts])
    flip = rng.random(ascii.size) < err
    ascii[flip] = rng.choice(np.frombuffer(b"ACGTN", np.uint8), int(flip.sum()))
    qual = rng.integers(2, 42, ascii.size).astype(np.uint8)
    return ascii, qual, np.arange(n + 1, dtype=np.int64) * L


@pytest.mark.parametrize("k,L", [(1, 4), (5, 12), (21, 100), (31, 31), (33, 40), (51, 150), (63, 200),
                                 (15, 16384 - 64)])
def test_stream_fixed_reads_every_owner(k, L):
    """Fixed-length reads: every owner of 3, with N bases, low-quality neighbours, runs of windows cut
    short at read ends (fewer than 8, exactly 8, one, not a multiple of 8 windows per read), 2k just
    above 64 bits and one read per tile; the stream holds exactly the owned windows (plus holes)."""
    n = max(3, 300_000 // L)
    ascii, qual, off = fixed_reads(2000 + k, k, L, n)
    total = 0
    for owner in range(3):
        got, exp = both(ascii, qual, off, k, read_len=L, qcut=25, n_owners=3, owner=owner)
        assert_tables_equal(got, exp, "stream, owner %d of 3, k=%d L=%d" % (owner, k, L))
        assert got["occ_entries"] >= got["card_positions"] == got["stats"]["occurrences"]
        total += len(got["count"])
    assert total == len(oracle.run(ascii, qual, off, k, qcut=25, n_threads=4)["count"])


@pytest.mark.parametrize("k", [1, 5, 21, 33, 51, 63])
def test_stream_variable_length_reads(k):
    """Ragged reads (0..220 bp, N and lowercase bases) take the offset path of the card pass."""
    ascii, qual, off = random_read_set(300 + k, 3000, 0, 220, genome_len=30000, n_rate=0.002, lower_rate=0.01)
    for n_owners, owner in ((1, 0), (4, 3)):
        got, exp = both(ascii, qual, off, k, qcut=20, n_owners=n_owners, owner=owner)
        assert_tables_equal(got, exp, "stream var k=%d owner %d of %d" % (k, owner, n_owners))


def test_stream_every_window_tiny_workload():
    """No owner filter: the stream holds every window of the tiny workload (1 Mbp, 200k x 100 bp)."""
    w = synth.tiny()
    r = w.reads()
    p = w.params
    got, exp = both(r.ascii, r.qual, r.offsets(), p.k, read_len=r.read_len, qcut=p.qcut, min_depth=p.min_depth)
    assert_tables_equal(got, exp, "stream tiny")
    assert got["digest"] == table_digest(exp)
    assert got["card_positions"] == r.n_reads * (r.read_len - p.k + 1)


@pytest.mark.parametrize("variant", ["forward_only", "bypass", "min_depth_1", "separate_bloom", "ext_min_3"])
def test_stream_variants(variant):
    ascii, qual, off = fixed_reads(77, 21, 100, 4000, genome_len=15000)
    kw = dict(qcut=20, n_owners=2, owner=1)
    okw = dict(kw)
    if variant == "forward_only":
        kw["forward_only"] = okw["forward_only"] = True
    elif variant == "bypass":
        kw["bypass"] = True
    elif variant == "min_depth_1":
        kw["min_depth"] = okw["min_depth"] = 1
    elif variant == "separate_bloom":
        kw["bloom_in_table"] = False
    else:
        kw["ext_min"] = okw["ext_min"] = 3
    got = kmer.analyze(ascii, qual, 21, read_len=100, occ_stream=True, **kw)
    exp = oracle.run(ascii, qual, off, 21, n_threads=4, **okw)
    assert_tables_equal(got, exp, "stream %s" % variant)


def test_stream_heavy_hitters():
    """Heavy keys found by the card pass are counted in workgroup-local memory by the stream pass too."""
    rng = np.random.default_rng(5)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 20000)
    L, n = 100, 6000
    reads = [g[s:s + L] for s in rng.integers(0, g.size - L + 1, n)]
    reads += [np.frombuffer(b"A" * L, np.uint8)] * 2000 + [np.frombuffer(b"CA" * (L // 2), np.uint8)] * 1000
    ascii = np.concatenate(reads)
    qual = rng.integers(2, 42, ascii.size).astype(np.uint8)
    off = np.arange(len(reads) + 1, dtype=np.int64) * L
    for n_owners, owner in ((1, 0), (2, 0), (2, 1)):
        got = kmer.analyze(ascii, qual, 31, read_len=L, occ_stream=True, n_owners=n_owners, owner=owner)
        exp = oracle.run(ascii, qual, off, 31, n_owners=n_owners, owner=owner, n_threads=4)
        assert_tables_equal(got, exp, "stream heavy, owner %d of %d" % (owner, n_owners))
        if n_owners == 1:
            assert got["n_heavy"] > 0 and got["stats"]["heavy_local"] > 0


def test_stream_matches_read_pass():
    """The stream pass and the pass over the reads give the same table and the same occurrence count."""
    ascii, qual, off = fixed_reads(9, 51, 150, 6000, genome_len=40000)
    a = kmer.analyze(ascii, qual, 51, read_len=150, n_owners=4, owner=2)
    b = kmer.analyze(ascii, qual, 51, read_len=150, n_owners=4, owner=2, occ_stream=True)
    assert_tables_equal(a, b, "reads vs stream")
    assert a["digest"] == b["digest"]
    assert a["stats"]["occurrences"] == b["stats"]["occurrences"]


def test_stream_overflow_is_reported_and_regrown():
    """A stream too small for the owned windows: the card pass drops entries past the capacity and
    pass 1 refuses the stream (HM_ST_STREAM_FULL -> HM_ECAPACITY); analyze() then regrows it and
    the result is exact."""
    ascii, qual, off = fixed_reads(11, 21, 100, 3000)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(ascii).to(dev)
    q = torch.from_numpy(qual).to(dev)
    packed = kmer.pack_reads(a, q, read_len=100, qcut=20)
    sk = kmer.CardSketch(21, packed.positions(21), n_owners=2, owner=0, device=dev)
    occ = kmer.OccStream(1000, device=dev)
    card = sk.run([packed], occ=occ)
    assert occ.overflowed() and card.positions > 1000
    cap, bw, lcap = kmer.plan_sizes(card, device=dev)
    kc = kmer.KmerCounter(21, cap, bw, lcap, n_owners=2, owner=0, device=dev)
    out = kmer.Records(kc.capacity, device=dev)
    kc.run_occ(occ, out, fused=True)
    assert kc.status() == abi.HM_ECAPACITY
    assert int(kc.status_buf.item()) & abi.HM_ST_STREAM_FULL
    assert "stream" in abi.last_error()
    got = kmer.analyze(ascii, qual, 21, read_len=100, n_owners=2, owner=0, occ_stream=True, occ_capacity=1000)
    exp = oracle.run(ascii, qual, off, 21, n_owners=2, owner=0)
    assert_tables_equal(got, exp, "regrown stream")


def test_stream_human_share_batches():
    """The human-scale share's recipe (interspersed repeats, owner 0 of 16) at 1/200 scale in four
    batches: one stream over all batches, one pass-1 launch over it, against the oracle."""
    w = synth.human_share(scale=1 / 200)
    p = w.params
    dev = torch.device("cuda:0")
    n = w.n_reads
    cuts = [0, n // 5, n // 2, (4 * n) // 5, n]
    host, packs = [], []
    for i in range(4):
        r = w.reads(r0=cuts[i], n=cuts[i + 1] - cuts[i])
        host.append(r)
        packs.append(kmer.pack_reads(torch.from_numpy(r.ascii).to(dev), torch.from_numpy(r.qual).to(dev),
                                     read_len=r.read_len, qcut=p.qcut))
    sk = kmer.CardSketch(p.k, w.positions, n_owners=p.n_owners, owner=p.owner, device=dev)
    occ = kmer.OccStream.for_windows(w.positions, p.n_owners, len(packs), device=dev)
    card = sk.run(packs, min_depth=p.min_depth, occ=occ)
    assert card.status == abi.HM_OK and not occ.overflowed()
    cap, bw, lcap = kmer.plan_sizes(card, device=dev)
    kc = kmer.KmerCounter(p.k, cap, bw, lcap, n_owners=p.n_owners, owner=p.owner, heavy=card, device=dev)
    out = kmer.Records(kc.capacity, device=dev)
    kc.run_occ(occ, out, fused=True)
    assert kc.status() == abi.HM_OK
    assert kc.stats()["occurrences"] == card.positions
    got = out.to_numpy()
    ascii = np.concatenate([r.ascii for r in host])
    qual = np.concatenate([r.qual for r in host])
    off = np.arange(n + 1, dtype=np.int64) * w.read_len
    exp = oracle.run(ascii, qual, off, p.k, qcut=p.qcut, n_owners=p.n_owners, owner=p.owner, n_threads=THREADS,
                     split_reads=True)
    assert_tables_equal(got, exp, "human share 1/200 via the stream")
    assert out.digest_words() == table_digest(exp)
    # the stream's entries: every owned window once, the rest holes
    e = occ.ext[:occ.entries()].cpu().numpy()
    assert int((e != 0xFF).sum()) == card.positions
