"""GPU path (through the C ABI) against the CPU oracle, record by record.

Integer output, so the bar is bit-exact equality of the sorted tables:
keys, counts, both tally arrays and both class bytes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, enc, pack_reads, random_read_set, read_golden, table_digest, table_to_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def both(ascii, qual, off, k, read_len=None, n_threads=4, **kw):
    okw = {x: kw[x] for x in ("qcut", "min_depth", "ext_min", "n_owners", "owner", "qual_offset", "forward_only")
           if x in kw}
    gkw = dict(kw)
    keep_all = gkw.pop("keep_all", False)
    if keep_all:
        gkw["export_flags"] = abi.HM_EXPORT_ALL
    got = kmer.analyze(ascii, qual, k, read_len=read_len, read_off=None if read_len else off, **gkw)
    exp = oracle.run(ascii, qual, off, k, keep_all=keep_all, n_threads=n_threads, **okw)
    return got, exp


# ------------------------------------------------------------------ pack layout

def numpy_pack(ascii, qual, qcut, qual_offset=0):
    """The layout documented at hm_reads_t, in numpy."""
    n = ascii.size
    nm_words = n // 64 + 3
    x = ascii | 0x20
    code = np.select([x == ord("c"), x == ord("g"), x == ord("t")], [1, 2, 3], 0).astype(np.uint64)
    valid = np.isin(x, np.frombuffer(b"acgt", np.uint8))
    good = valid & (qual.astype(np.int64) - qual_offset >= qcut)
    code[~valid] = 0
    b2 = np.zeros(2 * nm_words, np.uint64)
    nm = np.full(nm_words, np.uint64(2 ** 64 - 1))
    hq = np.zeros(nm_words, np.uint64)
    i = np.arange(n)
    np.bitwise_or.at(b2, i // 32, code << (62 - 2 * (i % 32)).astype(np.uint64))
    nm[: (n + 63) // 64] = 0
    tail = (n + 63) // 64 * 64
    if n % 64:
        j = np.arange(n, tail)
        np.bitwise_or.at(nm, j // 64, np.uint64(1) << (63 - j % 64).astype(np.uint64))
    np.bitwise_or.at(nm, i // 64, (~valid).astype(np.uint64) << (63 - i % 64).astype(np.uint64))
    np.bitwise_or.at(hq, i // 64, good.astype(np.uint64) << (63 - i % 64).astype(np.uint64))
    return b2, nm, hq


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000 + 37, 4096])
@pytest.mark.parametrize("offset", [0, 1])
def test_pack_layout(n, offset):
    rng = np.random.default_rng(n)
    ascii = rng.choice(np.frombuffer(b"ACGTNacgtX", np.uint8), n + offset)
    qual = rng.integers(0, 60, n + offset).astype(np.uint8)
    a = torch.from_numpy(ascii).cuda()[offset:]  # offset 1 exercises the unaligned load path
    q = torch.from_numpy(qual).cuda()[offset:]
    p = kmer.pack_reads(a, q, read_len=max(n, 1), qcut=20, qual_offset=3)
    torch.cuda.synchronize()
    b2, nm, hq = numpy_pack(ascii[offset:], qual[offset:], 20, 3)
    assert np.array_equal(p.bases2.cpu().numpy().view(np.uint64), b2)
    assert np.array_equal(p.nmask.cpu().numpy().view(np.uint64), nm)
    assert np.array_equal(p.hqmask.cpu().numpy().view(np.uint64), hq)


# ------------------------------------------------------------------ workloads

def test_tiny_workload_full_size():
    """The tiny workload at full size: 1 Mbp genome, 200k x 100 bp reads, k=21."""
    w = synth.tiny()
    r = w.reads()
    got, exp = both(r.ascii, r.qual, r.offsets(), 21, read_len=100, n_threads=8)
    assert_tables_equal(got, exp, "tiny")
    assert got["digest"] == table_digest(exp)
    assert len(exp["count"]) > 900_000


def test_mid_workload_scaled():
    """The mid workload's shape (repeats, end-biased errors, 150 bp, k=51) at 1/200 size."""
    w = synth.mid(scale=0.005)
    r = w.reads()
    got, exp = both(r.ascii, r.qual, r.offsets(), 51, read_len=150, n_threads=8)
    assert_tables_equal(got, exp, "mid/200")


@pytest.mark.parametrize("k", [1, 3, 5, 15, 21, 31, 33, 47, 51, 63])
def test_variable_length_reads_all_k(k):
    """Ragged reads (0..220 bp) with N and lowercase bases, several tiles, every key width."""
    ascii, qual, off = random_read_set(k, 3000, 0, 220, genome_len=30000, n_rate=0.002, lower_rate=0.01)
    got, exp = both(ascii, qual, off, k, qcut=20)
    assert_tables_equal(got, exp, "var k=%d" % k)


@pytest.mark.parametrize("k,L", [(21, 100), (31, 150), (51, 150), (63, 64), (5, 16384 - 64), (9, 20000)])
def test_fixed_length_reads(k, L):
    """Fixed-length reads (LDS-tiled path, ragged last tile; L above the tile size takes the
    offset path)."""
    n = max(3, 700_000 // L)
    rng = np.random.default_rng(L)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 40000)
    starts = rng.integers(0, g.size - L + 1, n)
    ascii = np.concatenate([g[s:s + L] for s in starts])
    flip = rng.random(ascii.size) < 0.01
    ascii[flip] = rng.choice(np.frombuffer(b"ACGTN", np.uint8), int(flip.sum()))
    qual = rng.integers(2, 42, ascii.size).astype(np.uint8)
    off = np.arange(n + 1, dtype=np.int64) * L
    if L <= 16384 - 64:
        got, exp = both(ascii, qual, off, k, read_len=L, qcut=25, min_depth=2, ext_min=3)
    else:
        got, exp = both(ascii, qual, off, k, qcut=25, min_depth=2, ext_min=3)
    assert_tables_equal(got, exp, "fixed k=%d L=%d" % (k, L))


@pytest.mark.parametrize("k,L", [(1, 4), (5, 12), (21, 100), (31, 31), (33, 40), (51, 150), (63, 200),
                                 (15, 16384 - 64)])
def test_owner_filtered_fixed_reads(k, L):
    """Fixed-length reads with an owner filter take the queued pass 1 (k_pass1_owned: each
    workgroup queues its owned occurrences in LDS and counts them 256 at a time with every lane
    busy): every owner of 3 against the oracle, with N bases, low-quality bases, few windows per
    read (L - k + 1 below 8, exactly 8, one, not a multiple of 8), 2k just above 64 bits, one read
    per tile; and forward-only keys."""
    n = max(3, 300_000 // L)
    rng = np.random.default_rng(1000 + k)
    g = rng.choice(np.frombuffer(b"ACGT", np.uint8), 20000)
    starts = rng.integers(0, g.size - L + 1, n)
    ascii = np.concatenate([g[s:s + L] for s in starts])
    flip = rng.random(ascii.size) < 0.01
    ascii[flip] = rng.choice(np.frombuffer(b"ACGTN", np.uint8), int(flip.sum()))
    qual = rng.integers(2, 42, ascii.size).astype(np.uint8)
    off = np.arange(n + 1, dtype=np.int64) * L
    total = 0
    for owner in range(3):
        got, exp = both(ascii, qual, off, k, read_len=L, qcut=25, n_owners=3, owner=owner)
        assert_tables_equal(got, exp, "owner %d of 3, k=%d L=%d" % (owner, k, L))
        total += len(got["count"])
    assert total == len(oracle.run(ascii, qual, off, k, qcut=25, n_threads=4)["count"])
    got, exp = both(ascii, qual, off, k, read_len=L, qcut=25, n_owners=2, owner=1, forward_only=True)
    assert_tables_equal(got, exp, "forward only, owner 1 of 2, k=%d L=%d" % (k, L))


@pytest.mark.parametrize("k", [5, 31, 51, 63])
def test_separate_bloom_filter(k):
    """The separate 64-bit-word filter (the table's classification words left out of pass 1):
    ragged reads, fixed-length reads with heavy hitters, and forward-only keys."""
    ascii, qual, off = random_read_set(100 + k, 3000, 0, 220, genome_len=30000, n_rate=0.002, lower_rate=0.01)
    got, exp = both(ascii, qual, off, k, qcut=20, bloom_in_table=False)
    assert_tables_equal(got, exp, "separate filter, var k=%d" % k)
    ascii, qual, off = random_read_set(200 + k, 2000, 150, 150, genome_len=8000)
    got, exp = both(ascii, qual, off, k, read_len=150, qcut=20, bloom_in_table=False)
    assert_tables_equal(got, exp, "separate filter, fixed k=%d" % k)
    assert got["n_heavy"] > 0 or k == 5  # the 8 kbp genome at 37x has k-mers frequent enough to be heavy
    got, exp = both(ascii, qual, off, k, read_len=150, qcut=20, bloom_in_table=False, forward_only=True)
    assert_tables_equal(got, exp, "separate filter, forward only k=%d" % k)


# ------------------------------------------------------------------ Bloom independence

@pytest.mark.parametrize("bloom_words,n_hash", [(1, 1), (1, 8), (64, 2), (1 << 22, 4)])
def test_output_independent_of_bloom(bloom_words, n_hash):
    """A 1-word separate filter makes nearly every first occurrence a false positive; a huge one
    almost none.  The table must not change."""
    ascii, qual, off = random_read_set(77, 2000, 90, 150, genome_len=15000)
    exp = oracle.run(ascii, qual, off, 31, n_threads=4)
    got = kmer.analyze(ascii, qual, 31, read_off=off, bloom_words=bloom_words, n_hash=n_hash, bloom_in_table=False)
    assert_tables_equal(got, exp, "bloom %d/%d" % (bloom_words, n_hash))


@pytest.mark.parametrize("capacity,n_hash", [(None, 1), (None, 8), (1024, 8), (1 << 20, 4)])
def test_output_independent_of_bloom_in_table(capacity, n_hash):
    """The filter in the table's classification words (32 bits per slot): planned sizes, a
    1024-slot start that fills up and is doubled until every kept k-mer and false positive
    fits, and a 2^20-slot table whose filter almost never errs.  The table must not change."""
    ascii, qual, off = random_read_set(77, 2000, 90, 150, genome_len=15000)
    exp = oracle.run(ascii, qual, off, 31, n_threads=4)
    got = kmer.analyze(ascii, qual, 31, read_off=off, capacity=capacity, bloom_words=1, n_hash=n_hash,
                       retries=8)
    assert_tables_equal(got, exp, "bloom in table, capacity %s, %d hashes" % (capacity, n_hash))
    st = got["stats"]
    assert 0 < st["deferred"] <= st["bloom_tests"]


@pytest.mark.parametrize("in_table", [True, False])
def test_classify_between_pass1_batches(in_table):
    """A classification between two pass-1 batches overwrites the classification words, which
    hold the filter when it is in the table: the classification marks the table, and the second
    batch then inserts every absent k-mer instead of testing the lost bits.  Either way the table
    equals the oracle's over both batches."""
    ascii, qual, off = random_read_set(15, 3000, 150, 150)
    exp = oracle.run(ascii, qual, off, 31)
    kc = kmer.KmerCounter(31, 1 << 17, 1 << 14, 1 << 19, bloom_in_table=in_table)
    assert kc.bloom_in_table == in_table
    packs = []
    for b0, b1 in ((0, 1400), (1400, 3000)):
        a0, a1 = off[b0], off[b1]
        packs.append(kmer.pack_reads(torch.from_numpy(ascii[a0:a1]).cuda(), torch.from_numpy(qual[a0:a1]).cuda(),
                                     read_len=150))
    out = kmer.Records(1 << 17)
    kc.reset()
    kc.insert(packs[0])
    deferred_1 = kc.stats()["deferred"]
    kc.classify()
    assert int(kc.status_buf.item()) == abi.HM_ST_CLASSIFIED
    kc.insert(packs[1])
    deferred_2 = kc.stats()["deferred"] - deferred_1
    kc.count()
    kc.export(out, abi.HM_EXPORT_CLASSIFY)
    assert kc.status() == abi.HM_OK
    assert_tables_equal(out.to_numpy(), exp, "classify between pass-1 batches")
    assert deferred_1 > 0
    if in_table:  # nothing of the second batch was deferred
        assert deferred_2 == 0
    else:
        assert deferred_2 > 0


def test_bypass_and_keep_all_sum():
    ascii, qual, off = random_read_set(5, 1500, 0, 200, n_rate=0.01)
    got, exp = both(ascii, qual, off, 21, bypass=True, keep_all=True, min_depth=2)
    assert_tables_equal(got, exp, "bypass+all")
    valid = oracle.run(ascii, qual, off, 21, keep_all=True, min_depth=1)["positions"]
    assert int(got["count"].astype(np.int64).sum()) == valid
    got1, exp1 = both(ascii, qual, off, 21, min_depth=1)
    assert_tables_equal(got1, exp1, "min_depth=1")


@pytest.mark.parametrize("seed", [1, 2, 0xDEADBEEF])
def test_output_independent_of_hash_seed_and_probe(seed):
    ascii, qual, off = random_read_set(9, 1500, 100, 150)
    exp = oracle.run(ascii, qual, off, 51)
    got = kmer.analyze(ascii, qual, 51, read_off=off, seed=seed, capacity=1 << 16)
    assert_tables_equal(got, exp, "seed %x" % seed)


# ------------------------------------------------------------------ paper examples, filters

def test_paper_examples_forward_only():
    g = read_golden("traversal_ctg.txt")
    reads = g["reads"][0]
    ascii = np.frombuffer("".join(reads).encode(), np.uint8).copy()
    qual = np.full(ascii.size, 40, np.uint8)
    got = kmer.analyze(ascii, qual, 3, read_len=len(reads[0]), forward_only=True, qcut=0)
    d = table_to_dict(got)
    uu = {key for key, v in d.items() if v[3] < 4 and v[4] < 4}
    assert uu == {enc(x) for x in g["uu"][0]}
    cnt, tl, tr, cl, cr = d[enc("CTG")]
    assert (cr, cl) == (0, 3)  # right A, left T
    f = read_golden("fork_gaa.txt")
    ascii = np.frombuffer("".join(f["reads"][0]).encode(), np.uint8).copy()
    got = kmer.analyze(ascii, np.full(ascii.size, 40, np.uint8), 3, read_len=4, qcut=0)
    assert table_to_dict(got)[enc("GAA")][4] == abi.HM_CLS_FORK


def test_owner_filter_partition():
    ascii, qual, off = random_read_set(31, 2500, 120, 150)
    parts = []
    for p in range(4):
        got, exp = both(ascii, qual, off, 51, n_owners=4, owner=p)
        assert_tables_equal(got, exp, "owner %d" % p)
        parts.append(got)
    whole = oracle.run(ascii, qual, off, 51)
    assert sum(len(p["count"]) for p in parts) == len(whole["count"])


def test_uu_only_export():
    ascii, qual, off = random_read_set(41, 2000, 150, 150)
    got = kmer.analyze(ascii, qual, 31, read_off=off, export_flags=abi.HM_EXPORT_UU_ONLY)
    exp = oracle.run(ascii, qual, off, 31)
    m = oracle.uu_mask(exp)
    assert_tables_equal(got, {x: v[m] for x, v in exp.items() if isinstance(v, np.ndarray)}, "uu")


# ------------------------------------------------------------------ edge cases

def test_empty_and_degenerate_inputs():
    # no reads
    z = np.zeros(0, np.uint8)
    got = kmer.analyze(z, z, 21, read_off=np.zeros(1, np.int64))
    assert len(got["count"]) == 0
    # every read shorter than k, and all-N reads
    ascii, qual, off = random_read_set(3, 500, 0, 20)
    got, exp = both(ascii, qual, off, 21, keep_all=True, min_depth=1)
    assert len(got["count"]) == 0 == len(exp["count"])
    ascii = np.full(3000, ord("N"), np.uint8)
    got = kmer.analyze(ascii, np.full(3000, 40, np.uint8), 21, read_len=150, export_flags=abi.HM_EXPORT_ALL)
    assert len(got["count"]) == 0


def test_hot_key_contention():
    """One k-mer a million times (poly-A reads) plus normal reads: counts and tallies exact under
    same-address atomics from every wave."""
    ascii, qual, off = random_read_set(8, 1000, 150, 150)
    n_hot = 10_000
    hot = np.full(n_hot * 150, ord("A"), np.uint8)
    a2 = np.concatenate([ascii, hot])
    q2 = np.concatenate([qual, np.full(hot.size, 40, np.uint8)])
    off2 = np.concatenate([off, off[-1] + np.arange(1, n_hot + 1, dtype=np.int64) * 150])
    for k in (21, 51):
        got, exp = both(a2, q2, off2, k)
        assert_tables_equal(got, exp, "hot k=%d" % k)
        assert int(exp["count"][0]) >= n_hot * (150 - k + 1)


def test_capacity_errors_are_reported_not_wrong():
    ascii, qual, off = random_read_set(12, 2000, 150, 150)
    exp = oracle.run(ascii, qual, off, 31)
    # too small a table: the direct call reports HM_ECAPACITY
    kc = kmer.KmerCounter(31, 256, 1 << 12, 1 << 20, max_probe=32)
    a = torch.from_numpy(ascii).cuda()
    q = torch.from_numpy(qual).cuda()
    p = kmer.pack_reads(a, q, read_off=torch.from_numpy(off).cuda())
    out = kmer.Records(256)
    kc.run([p], out)
    assert kc.status() == abi.HM_ECAPACITY
    # too small a list, likewise
    kc = kmer.KmerCounter(31, 1 << 18, 1 << 12, 100)
    kc.run([p], out)
    assert kc.status() == abi.HM_ECAPACITY
    # the retrying driver grows both and gets the exact table
    got = kmer.analyze(ascii, qual, 31, read_off=off, capacity=1024, list_capacity=1000, max_probe=64, retries=12)
    assert_tables_equal(got, exp, "after retries")


def test_owner_filtered_capacity_errors():
    """A table that fills during owner-filtered pass 1 over fixed-length reads (the queued loop, whose
    workgroups notice a full table at their next tile and stop together, then count what they had
    queued) is reported as a capacity error; the retrying driver ends with the owner's exact table.
    250k reads make about 2300 tiles, more than the workgroups of one launch, so workgroups reach a
    later tile after the table has filled."""
    ascii, qual, off = random_read_set(13, 250_000, 150, 150, genome_len=200_000)
    exp = oracle.run(ascii, qual, off, 31, n_owners=2, owner=1, n_threads=8)
    a = torch.from_numpy(ascii).cuda()
    q = torch.from_numpy(qual).cuda()
    p = kmer.pack_reads(a, q, read_len=150)
    kc = kmer.KmerCounter(31, 256, 64, 1 << 24, n_owners=2, owner=1, max_probe=32)
    out = kmer.Records(1 << 16)
    kc.run([p], out)
    assert kc.status() == abi.HM_ECAPACITY
    assert int(kc.status_buf.item()) & abi.HM_ST_TABLE_FULL
    # a 1024-slot start (bloom_words=1 keeps the table from growing to the planned filter's size)
    got = kmer.analyze(ascii, qual, 31, read_len=150, n_owners=2, owner=1, capacity=1024, bloom_words=1,
                       max_probe=64, retries=12)
    assert_tables_equal(got, exp, "owner-filtered, after retries")
    assert got["capacity"] > 1024


def test_export_buffer_too_small():
    ascii, qual, off = random_read_set(13, 500, 150, 150)
    kc = kmer.KmerCounter(31, 1 << 16, 1 << 12, 1 << 18)
    p = kmer.pack_reads(torch.from_numpy(ascii).cuda(), torch.from_numpy(qual).cuda(),
                        read_off=torch.from_numpy(off).cuda())
    out = kmer.Records(10)
    kc.run([p], out)
    assert kc.status() == abi.HM_EOUTPUT
    need = int(out.n_out.item())
    assert need == len(oracle.run(ascii, qual, off, 31)["count"])


def test_batches_into_one_table():
    """Several pass-1 batches into one table (the streamed human-scale shape) equal one pass
    over all reads."""
    ascii, qual, off = random_read_set(14, 3000, 150, 150)
    exp = oracle.run(ascii, qual, off, 51)
    kc = kmer.KmerCounter(51, 1 << 17, 1 << 14, 1 << 19)
    cuts = [0, 700, 1900, 3000]
    packs = []
    for i in range(3):
        b0, b1 = off[cuts[i]], off[cuts[i + 1]]
        packs.append(kmer.pack_reads(torch.from_numpy(ascii[b0:b1]).cuda(), torch.from_numpy(qual[b0:b1]).cuda(),
                                     read_len=150))
    out = kmer.Records(1 << 17)
    kc.run(packs, out)
    assert kc.status() == abi.HM_OK
    assert_tables_equal(out.to_numpy(), exp, "batched pass 1")


@pytest.mark.parametrize("k", [21, 51])
def test_fused_classify_export_and_presence_filter(k):
    """Classification fused into the export sweep, and the pass-2 presence filter switched off,
    give the same table as the separate classify call and the oracle."""
    ascii, qual, off = random_read_set(60 + k, 3000, 100, 150, genome_len=40000)
    exp = oracle.run(ascii, qual, off, k, n_threads=4)
    for fused in (False, True):
        for pf in (True, False):
            got = kmer.analyze(ascii, qual, k, read_off=off, fused=fused, present_filter=pf)
            assert_tables_equal(got, exp, "fused=%s filter=%s" % (fused, pf))
    a = kmer.analyze(ascii, qual, k, read_off=off, fused=True, export_flags=abi.HM_EXPORT_UU_ONLY)
    b = kmer.analyze(ascii, qual, k, read_off=off, fused=False, export_flags=abi.HM_EXPORT_UU_ONLY)
    assert_tables_equal(a, b, "uu only")
    # HM_EXPORT_ALL also returns the Bloom false-positive singletons, a set that depends on the
    # order occurrences reach the filter: compare what is unique (count >= 2), and check that
    # every count-1 record is a true singleton of the input
    single = oracle.run(ascii, qual, off, k, keep_all=True, min_depth=1, n_threads=4)
    singles = set(zip(single["key_hi"][single["count"] == 1].tolist(), single["key_lo"][single["count"] == 1].tolist()))
    for fused in (True, False):
        t = kmer.analyze(ascii, qual, k, read_off=off, fused=fused, export_flags=abi.HM_EXPORT_ALL)
        m = t["count"] >= 2
        assert_tables_equal({x: v[m] for x, v in t.items() if isinstance(v, np.ndarray)}, exp, "all, count >= 2")
        ones = set(zip(t["key_hi"][~m].tolist(), t["key_lo"][~m].tolist()))
        assert (t["count"][~m] == 1).all() and ones <= singles


# ------------------------------------------------------------------ key-ordered export

@pytest.mark.parametrize("k", [1, 5, 15, 17, 21, 31, 33, 37, 51, 63])
def test_sorted_export_order(k):
    """HM_EXPORT_SORTED: the device's record order is the oracle's key order, record by record
    (many tiles, a ragged last tile, 1 to 16 radix passes, one- and two-word keys)."""
    ascii, qual, off = random_read_set(500 + k, 3000, 0, 220, genome_len=30000, n_rate=0.002, lower_rate=0.01)
    exp = oracle.run(ascii, qual, off, k, n_threads=4)
    for fused in (False, True):
        got = kmer.analyze(ascii, qual, k, read_off=off, export_flags=abi.HM_EXPORT_SORTED, fused=fused)
        assert_tables_equal(got, exp, "sorted k=%d fused=%s" % (k, fused))
        plain = kmer.analyze(ascii, qual, k, read_off=off, fused=fused)
        assert got["digest"] == plain["digest"]


@pytest.mark.parametrize("k", [2, 16, 32])
def test_sorted_export_forward_only_even_k(k):
    """Forward-only keys of exactly 64 bits (k=32) and a 4-bit key (k=2)."""
    ascii, qual, off = random_read_set(700 + k, 2000, 40, 150, genome_len=20000)
    exp = oracle.run(ascii, qual, off, k, forward_only=True, n_threads=4)
    got = kmer.analyze(ascii, qual, k, read_off=off, forward_only=True, export_flags=abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, exp, "sorted forward k=%d" % k)


def test_sorted_export_workload_scale():
    """The tiny workload at full size (about a million records, 6 passes) and the mid workload's
    shape at 1/200 (k=51, 13 passes), sorted on the device."""
    w = synth.tiny()
    r = w.reads()
    exp = oracle.run(r.ascii, r.qual, r.offsets(), 21, n_threads=8)
    got = kmer.analyze(r.ascii, r.qual, 21, read_len=100, fused=True, export_flags=abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, exp, "tiny sorted")
    w = synth.mid(scale=0.005)
    r = w.reads()
    exp = oracle.run(r.ascii, r.qual, r.offsets(), 51, n_threads=8)
    got = kmer.analyze(r.ascii, r.qual, 51, read_len=150, fused=True, export_flags=abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, exp, "mid/200 sorted")


def test_sorted_export_with_other_flags():
    ascii, qual, off = random_read_set(811, 3000, 100, 150, genome_len=40000)
    exp = oracle.run(ascii, qual, off, 31, n_threads=4)
    m = oracle.uu_mask(exp)
    got = kmer.analyze(ascii, qual, 31, read_off=off, export_flags=abi.HM_EXPORT_UU_ONLY | abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, {x: v[m] for x, v in exp.items() if isinstance(v, np.ndarray)}, "uu sorted")
    # every slot: keys strictly increasing, and the part that is unique (count >= 2) equal to the oracle's
    got = kmer.analyze(ascii, qual, 31, read_off=off, export_flags=abi.HM_EXPORT_ALL | abi.HM_EXPORT_SORTED)
    key = got["key_hi"].astype(object) * 2 ** 64 + got["key_lo"].astype(object)
    assert all(a < b for a, b in zip(key[:-1], key[1:]))
    keep = got["count"] >= 2
    assert_tables_equal({x: v[keep] for x, v in got.items() if isinstance(v, np.ndarray)}, exp, "all sorted")


def test_sorted_export_empty_and_too_small():
    z = np.zeros(0, np.uint8)
    got = kmer.analyze(z, z, 21, read_off=np.zeros(1, np.int64), export_flags=abi.HM_EXPORT_SORTED)
    assert len(got["count"]) == 0
    # an export buffer too small reports HM_EOUTPUT (the partial records are sorted but invalid);
    # the same table then exports in full, in key order
    ascii, qual, off = random_read_set(812, 2000, 100, 150, genome_len=30000)
    exp = oracle.run(ascii, qual, off, 21, n_threads=4)
    a = torch.from_numpy(ascii).cuda()
    q = torch.from_numpy(qual).cuda()
    packed = kmer.pack_reads(a, q, read_off=torch.from_numpy(off).cuda(), qcut=20)
    kc = kmer.KmerCounter(21, 1 << 18, 1 << 14, 1 << 20, device="cuda")
    small = kmer.Records(100, device="cuda")
    kc.run([packed], small, flags=abi.HM_EXPORT_SORTED, fused=True)
    assert kc.status() == abi.HM_EOUTPUT
    assert int(small.n_out.item()) == len(exp["count"])
    full = kmer.Records(len(exp["count"]) + 10, device="cuda")
    kc.status_buf.zero_()
    kc.export(full, abi.HM_EXPORT_SORTED | abi.HM_EXPORT_CLASSIFY)
    assert kc.status() == abi.HM_OK
    assert_tables_equal(full.to_numpy(sort=False), exp, "after resize")


@pytest.mark.parametrize("k", [21, 37, 51])
def test_sorted_export_large_prefix_group(k):
    """More than 4096 distinct k-mers sharing their first 8 bases (one 16-bit prefix group larger
    than a workgroup sorts in LDS) among ordinary reads: the fallback path keeps the exact order."""
    rng = np.random.default_rng(3000 + k)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    special = [np.concatenate([np.full(8, ord("A"), np.uint8), rng.choice(acgt, k - 8)]) for _ in range(6000)]
    g = rng.choice(acgt, 40000)
    st = rng.integers(0, g.size - 120, 4000)
    reads = special + special + [g[s:s + 120] for s in st]  # every special k-mer twice: count 2, kept
    ascii = np.concatenate(reads)
    lens = np.array([len(r) for r in reads])
    off = np.zeros(len(reads) + 1, np.int64)
    off[1:] = np.cumsum(lens)
    qual = np.full(ascii.size, 40, np.uint8)
    exp = oracle.run(ascii, qual, off, k, n_threads=4)
    got = kmer.analyze(ascii, qual, k, read_off=off, export_flags=abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, exp, "large group k=%d" % k)
    pref = (exp["key_hi"].astype(object) * 2 ** 64 + exp["key_lo"].astype(object)) >> (2 * k - 16)
    assert (pref == 0).sum() > 4096


@pytest.mark.parametrize("k", [31, 51])
def test_sorted_export_tie_runs(k):
    """Keys sharing their first 20 bases (the 16-bit prefix and the next 24 bits): a run of 40 is
    ordered by the insertion step, a run of 100 sends its group through the general path."""
    rng = np.random.default_rng(4000 + k)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    p1 = np.frombuffer(b"AAAACCCCGGGGTTTTACGT", np.uint8)
    p2 = np.frombuffer(b"CCCCAAAATTTTGGGGTGCA", np.uint8)
    special = [np.concatenate([p1, rng.choice(acgt, k - 20)]) for _ in range(40)]
    special += [np.concatenate([p2, rng.choice(acgt, k - 20)]) for _ in range(100)]
    g = rng.choice(acgt, 30000)
    st = rng.integers(0, g.size - 100, 3000)
    reads = special + special + [g[s:s + 100] for s in st]
    ascii = np.concatenate(reads)
    off = np.zeros(len(reads) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in reads])
    qual = np.full(ascii.size, 40, np.uint8)
    exp = oracle.run(ascii, qual, off, k, forward_only=True, n_threads=4)
    got = kmer.analyze(ascii, qual, k, read_off=off, forward_only=True, export_flags=abi.HM_EXPORT_SORTED)
    assert_tables_equal(got, exp, "tie runs k=%d" % k)


@pytest.mark.parametrize("k,n_keys", [(21, 58), (51, 60), (31, 64)])
def test_nearly_full_small_table(k, n_keys):
    """A 64-slot table filled to 90-100% (every k-mer inserted, Bloom bypassed): long probe sequences
    that run through several lines and wrap past the end of the table; the table is exact, and one
    key more than the slots is reported as a full table."""
    rng = np.random.default_rng(k * 7 + n_keys)
    g = "".join(rng.choice(list("ACGT"), n_keys + k - 1))  # n_keys distinct k-mers (checked below)
    seqs = [g] * 3
    a, q, off = pack_reads([(s, [40] * len(s)) for s in seqs])
    exp = oracle.run(a, q, off, k, qcut=0, keep_all=True, min_depth=1)
    if len(exp["count"]) != n_keys:
        pytest.skip("the random genome repeats a k-mer")
    kc = kmer.KmerCounter(k, 64, 1, 0, min_depth=1, flags=abi.HM_BLOOM_BYPASS, max_probe=64)
    p = kmer.pack_reads(torch.from_numpy(a).cuda(), torch.from_numpy(q).cuda(), read_off=torch.from_numpy(off).cuda())
    out = kmer.Records(64)
    kc.run([p], out, flags=abi.HM_EXPORT_ALL, fused=True)
    if n_keys <= 64:
        assert kc.status() == abi.HM_OK
        assert_tables_equal(out.to_numpy(), exp, "64-slot table, %d keys" % n_keys)
    g2 = "".join(rng.choice(list("ACGT"), 64 + k))  # 65 distinct k-mers (or close): more than the slots
    a2, q2, off2 = pack_reads([(g2, [40] * len(g2))] * 2)
    if len(oracle.run(a2, q2, off2, k, qcut=0, keep_all=True, min_depth=1)["count"]) > 64:
        kc.run([kmer.pack_reads(torch.from_numpy(a2).cuda(), torch.from_numpy(q2).cuda(),
                                read_off=torch.from_numpy(off2).cuda())], out, flags=abi.HM_EXPORT_ALL, fused=True)
        assert kc.status() == abi.HM_ECAPACITY
