"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names what it pins.  None of them compares the oracle with itself:
the references are the paper's worked examples (tests/golden), a Python
brute force over string slices (tests/brute.py), closed forms and invariants.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests import brute
from tests.util import assert_tables_equal, enc, pack_reads, read_golden, table_to_dict

BASES = "ACGT"
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def ascending(t) -> bool:
    """Records in strictly ascending key order (the oracle's output contract)."""
    hi, lo = t["key_hi"], t["key_lo"]
    return bool(((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))).all())


def run_reads(reads, k, **kw):
    a, q, off = pack_reads(reads)
    t = oracle.run(a, q, off, k, **kw)
    assert ascending(t), "oracle output not in ascending key order"
    return t


def hq_reads(seqs, q=40):
    return [(s, [q] * len(s)) for s in seqs]


# ---------------------------------------------------------------- paper examples

def test_fig2b_chop_forward():
    """Figure 2(b): GATCTGAACCG with k=3 yields exactly its 9 overlapping 3-mers."""
    g = read_golden("fig2b_chop.txt")
    read, k = g["read"][0][0], int(g["k"][0][0])
    t = run_reads(hq_reads([read]), k, forward_only=True, keep_all=True, min_depth=1)
    d = table_to_dict(t)
    expected = g["kmers"][0]
    assert sorted(d) == sorted(enc(w) for w in expected)
    assert all(v[0] == 1 for v in d.values())
    assert t["positions"] == len(read) - k + 1 == len(expected)


def test_traversal_example_ctg():
    """Contig-generation example: CTG has value AT (right A, left T); UU = ATC, TCT, CTG;
    the right lookup from CTG is TGA."""
    g = read_golden("traversal_ctg.txt")
    k = int(g["k"][0][0])
    t = run_reads(hq_reads(g["reads"][0]), k, forward_only=True, qcut=0, min_depth=2, ext_min=2)
    d = table_to_dict(t)
    (kmer, _, rb, _, lb), = g["record"]
    cnt, tl, tr, cl, cr = d[enc(kmer)]
    assert cr == BASES.index(rb) and cl == BASES.index(lb)
    uu = {key for key, v in d.items() if v[3] < 4 and v[4] < 4}
    assert uu == {enc(w) for w in g["uu"][0]}
    for w in g["not_uu"][0]:
        assert enc(w) in d and enc(w) not in uu
    src, nxt = g["next_right"][0]
    assert enc(src[1:] + BASES[d[enc(src)][4]]) == enc(nxt)


@pytest.mark.parametrize("forward_only", [True, False])
def test_fork_gaa(forward_only):
    """De Bruijn graph example: GAA has two forward neighbours, so its right side is a fork
    (also in canonical mode: GAA < TTC keeps the forward orientation)."""
    g = read_golden("fork_gaa.txt")
    k = int(g["k"][0][0])
    t = run_reads(hq_reads(g["reads"][0]), k, forward_only=forward_only, qcut=0)
    d = table_to_dict(t)
    key = enc(g["fork_right"][0][0])
    assert d[key][4] == oracle.CLS_FORK
    assert d[key][2] == (0, 2, 0, 2)  # C twice, T twice


# ---------------------------------------------------------------- brute force (P1)

read_st = st.tuples(st.text(alphabet="ACGTNacgt", min_size=0, max_size=40), st.integers(0, 2 ** 31))


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(reads=st.lists(read_st, min_size=0, max_size=8), k=st.sampled_from([1, 3, 5, 7]),
       qcut=st.integers(0, 42), min_depth=st.integers(1, 3), ext_min=st.integers(1, 3),
       n_owners=st.sampled_from([1, 3]), fwd=st.booleans(), keep_all=st.booleans(),
       mode=st.sampled_from(["map", "split", "sort", "sort_threads"]))
def test_oracle_equals_brute_force(reads, k, qcut, min_depth, ext_min, n_owners, fwd, keep_all, mode):
    """Every counting scheme of the oracle (one map; read-partitioned maps; sort-counted, on one and
    on three threads) against the brute force."""
    kw = {"map": {}, "split": dict(n_threads=3, split_reads=True), "sort": dict(sort_count=True),
          "sort_threads": dict(sort_count=True, n_threads=3)}[mode]
    rs = []
    for s, seed in reads:
        rng = np.random.default_rng(seed)
        rs.append((s, [int(x) for x in rng.integers(0, 42, len(s))]))
    # repeat reads so that depth filters keep something
    rs = rs + rs[: len(rs) // 2]
    for own in range(n_owners):
        exp = brute.brute(rs, k, qcut=qcut, min_depth=min_depth, ext_min=ext_min, forward_only=fwd,
                          keep_all=keep_all, n_owners=n_owners, own=own)
        t = run_reads(rs, k, qcut=qcut, min_depth=min_depth, ext_min=ext_min, forward_only=fwd, keep_all=keep_all,
                      n_owners=n_owners, owner=own, **kw)
        assert table_to_dict(t) == exp


def test_brute_force_larger_k_and_threads():
    """k up to 63 (two 64-bit words) and the threaded oracle against the brute force."""
    rng = np.random.default_rng(5)
    g = "".join(rng.choice(list(BASES), 400))
    reads = []
    for _ in range(60):
        s = int(rng.integers(0, 400 - 90))
        r = g[s:s + 90]
        if rng.random() < 0.5:
            r = "".join(COMP[c] for c in reversed(r))
        reads.append((r, [int(x) for x in rng.integers(10, 41, 90)]))
    for k in (31, 33, 51, 63):
        exp = brute.brute(reads, k, qcut=20, min_depth=2)
        for T in (1, 3):
            assert table_to_dict(run_reads(reads, k, qcut=20, min_depth=2, n_threads=T)) == exp
            assert table_to_dict(run_reads(reads, k, qcut=20, min_depth=2, n_threads=T, split_reads=True)) == exp
            assert table_to_dict(run_reads(reads, k, qcut=20, min_depth=2, n_threads=T, sort_count=True)) == exp
        shard1 = {key: v for key, v in exp.items()
                  if oracle.shard_of(np.array([key >> 64], np.uint64),
                                     np.array([key & (2 ** 64 - 1)], np.uint64), 3)[0] == 1}
        got = run_reads(reads, k, qcut=20, min_depth=2, n_threads=4, split_reads=True, n_shards=3, shard=1)
        assert table_to_dict(got) == shard1
        got = run_reads(reads, k, qcut=20, min_depth=2, n_threads=4, sort_count=True, n_shards=3, shard=1)
        assert table_to_dict(got) == shard1


@pytest.mark.parametrize("mode", [dict(), dict(n_threads=2, split_reads=True), dict(sort_count=True),
                                  dict(n_threads=3, sort_count=True)])
def test_keys_sharing_their_low_word(mode):
    """Two-word keys (k = 33) that differ only in their first base share the low 64 key bits: keys
    must be told apart by both words (every scheme, against the brute force).  The reads alternate
    between the two k-mers so that no scheme sees them grouped by accident."""
    x = "GATTACAGATTACAGATTACAGATTACAGATT"  # 32 bases: the low 64 bits of both keys
    reads = []
    for i in range(12):
        reads.append((("A" if i % 2 else "C") + x + "G", [40] * 34))
    exp = brute.brute(reads, 33, qcut=20, min_depth=2, forward_only=True)
    got = run_reads(reads, 33, qcut=20, min_depth=2, forward_only=True, **mode)
    assert table_to_dict(got) == exp
    assert len(exp) == 3 and sorted(v[0] for v in exp.values()) == [6, 6, 12]


@pytest.mark.parametrize("mode", [dict(), dict(n_threads=3), dict(n_threads=3, split_reads=True),
                                  dict(sort_count=True), dict(n_threads=4, sort_count=True)])
def test_batched_reads_equal_brute_force(mode):
    """Reads given in batches (oracle.Accumulator) against the brute force over all of them: the
    unfiltered tables of the batches add up to the table of their union, and the depth filter and
    classes apply once at the end (a k-mer seen once in each of two batches is kept)."""
    rng = np.random.default_rng(17)
    g = "".join(rng.choice(list(BASES), 300))
    reads = []
    for _ in range(50):
        s = int(rng.integers(0, 300 - 60))
        r = g[s:s + 60]
        if rng.random() < 0.5:
            r = "".join(COMP[c] for c in reversed(r))
        reads.append((r, [int(x) for x in rng.integers(10, 41, 60)]))
    for k, owners in ((21, 1), (33, 2)):
        for own in range(owners):
            exp = brute.brute(reads, k, qcut=20, min_depth=2, n_owners=owners, own=own)
            acc = oracle.Accumulator(k, qcut=20, min_depth=2, n_owners=owners, owner=own, **mode)
            for lo, hi in ((0, 7), (7, 30), (30, 30), (30, 50)):
                a, q, off = pack_reads(reads[lo:hi])
                acc.add(a, q, off)
            got = acc.finish()
            assert ascending(got)
            assert table_to_dict(got) == exp
            assert got["positions"] == sum(len(r) - k + 1 for r, _ in reads)


def test_owner_map_matches_independent_python():
    """own(key) from the oracle equals a Python implementation of the same published finalizer."""
    rng = np.random.default_rng(1)
    hi = rng.integers(0, 2 ** 62, 500, dtype=np.uint64)
    lo = rng.integers(0, 2 ** 63, 500, dtype=np.uint64)
    o = oracle.owner_of(hi, lo, 16)
    for h, l, x in zip(hi, lo, o):
        assert brute.owner((int(h) << 64) | int(l), 16) == int(x)


@pytest.mark.parametrize("k,n", [(31, 16), (51, 16), (51, 5), (51, 1024)])
def test_owner_map_balances_a_genomes_kmers(k, n):
    """The owner map spreads the distinct canonical k-mers of a random 300 kbp genome (chains of
    keys that are shifts of one another, as every genome's are) evenly: the owner counts pass a
    chi-square test (n - 1 degrees of freedom, bound 6 standard deviations above the mean).  A map
    that used only part of the key, or left its top bits poorly mixed, fails it."""
    rng = np.random.default_rng(17 + k + n)
    g = "".join(rng.choice(list(BASES), 300_000))
    reads = [g[i:i + 150] for i in range(0, len(g) - 150 + 1, 100)]
    t = run_reads(hq_reads(reads), k, min_depth=1)
    N = len(t["count"])
    assert N > 290_000
    c = np.bincount(oracle.owner_of(t["key_hi"], t["key_lo"], n), minlength=n)
    assert len(c) == n
    e = N / n
    chi2 = float(((c - e) ** 2 / e).sum())
    assert chi2 < (n - 1) + 6 * (2 * (n - 1)) ** 0.5, chi2
    if n == 1024:  # owners nest for powers of two: owner j of 1024 lies inside owner j // 64 of 16
        o16 = oracle.owner_of(t["key_hi"], t["key_lo"], 16)
        assert (oracle.owner_of(t["key_hi"], t["key_lo"], 1024) // 64 == o16).all()


def test_invalid_arguments():
    a, q, off = pack_reads(hq_reads(["ACGT"]))
    with pytest.raises(ValueError):
        oracle.run(a, q, off, 4)  # even k in canonical mode
    with pytest.raises(ValueError):
        oracle.run(a, q, off, 65)
    with pytest.raises(ValueError):
        oracle.run(a, q, off, 3, n_owners=2, owner=2)


# ---------------------------------------------------------------- closed forms and invariants

def random_reads(rng, n, L_lo, L_hi, genome_len=3000, n_rate=0.0):
    g = "".join(rng.choice(list(BASES), genome_len))
    out = []
    for _ in range(n):
        L = int(rng.integers(L_lo, L_hi + 1))
        s = int(rng.integers(0, genome_len - L))
        r = list(g[s:s + L])
        if rng.random() < 0.5:
            r = [COMP[c] for c in reversed(r)]
        for j in range(L):
            if rng.random() < 0.01:
                r[j] = BASES[(BASES.index(r[j]) + int(rng.integers(1, 4))) % 4]
            if rng.random() < n_rate:
                r[j] = "N"
        out.append(("".join(r), [int(x) for x in rng.integers(2, 42, L)]))
    return out


def valid_windows(reads, k):
    n = 0
    for s, _ in reads:
        for i in range(len(s) - k + 1):
            if "N" not in s[i:i + k]:
                n += 1
    return n


@pytest.mark.parametrize("k", [5, 21, 51])
def test_count_sum_equals_valid_positions(k):
    """Sum of counts over the unfiltered table = number of valid windows (the Theta(Gd(L-k+1)/L)
    volume of the k-mer exchange, made exact)."""
    rng = np.random.default_rng(k)
    reads = random_reads(rng, 300, 0, 120, n_rate=0.005)
    t = run_reads(reads, k, keep_all=True, min_depth=1)
    assert int(t["count"].sum()) == valid_windows(reads, k) == t["positions"]


def test_tally_bounds_and_closed_form():
    """Each tally <= count; with Q=0 and no N, total tallies = 2 * sum(max(0, L - k))."""
    rng = np.random.default_rng(7)
    k = 21
    reads = random_reads(rng, 400, 10, 150)
    t = run_reads(reads, k, keep_all=True, min_depth=1, qcut=0)
    assert (t["tl"] <= t["count"][:, None]).all() and (t["tr"] <= t["count"][:, None]).all()
    assert (t["tl"].sum(1) <= t["count"]).all() and (t["tr"].sum(1) <= t["count"]).all()
    assert int(t["tl"].sum() + t["tr"].sum()) == 2 * sum(max(0, len(s) - k) for s, _ in reads)
    tq = run_reads(reads, k, keep_all=True, min_depth=1, qcut=20)
    assert int(tq["tl"].sum()) < int(t["tl"].sum())


def test_reverse_complement_invariance():
    """T(R) = T(rc(R)) when every read is reverse complemented and its qualities reversed."""
    rng = np.random.default_rng(11)
    reads = random_reads(rng, 300, 30, 150, n_rate=0.003)
    rc = [("".join(COMP.get(c, "N") for c in reversed(s)), list(reversed(q))) for s, q in reads]
    for k in (21, 51):
        a = run_reads(reads, k, keep_all=True, min_depth=1)
        b = run_reads(rc, k, keep_all=True, min_depth=1)
        assert_tables_equal(a, b, "rc k=%d" % k)


def test_permutation_and_additivity():
    """Read order does not matter, and unfiltered tables add: T(R u R') = T(R) + T(R')."""
    rng = np.random.default_rng(12)
    reads = random_reads(rng, 400, 40, 150)
    k = 31
    whole = table_to_dict(run_reads(reads, k, keep_all=True, min_depth=1))
    perm = [reads[i] for i in rng.permutation(len(reads))]
    assert table_to_dict(run_reads(perm, k, keep_all=True, min_depth=1)) == whole
    a = table_to_dict(run_reads(reads[:150], k, keep_all=True, min_depth=1))
    b = table_to_dict(run_reads(reads[150:], k, keep_all=True, min_depth=1))
    merged = {}
    for d in (a, b):
        for key, (c, tl, tr, _, _) in d.items():
            m = merged.setdefault(key, [0, [0] * 4, [0] * 4])
            m[0] += c
            m[1] = [x + y for x, y in zip(m[1], tl)]
            m[2] = [x + y for x, y in zip(m[2], tr)]
    assert {key: (v[0], tuple(v[1]), tuple(v[2])) for key, v in merged.items()} == \
        {key: v[:3] for key, v in whole.items()}


def test_owner_partition_union():
    """Union over owners of the owner-filtered tables = the unfiltered table, with disjoint keys."""
    rng = np.random.default_rng(13)
    reads = random_reads(rng, 500, 100, 150)
    k = 51
    whole = run_reads(reads, k)
    parts = [run_reads(reads, k, n_owners=5, owner=p) for p in range(5)]
    keys = [set(table_to_dict(p)) for p in parts]
    assert sum(len(s) for s in keys) == len(set().union(*keys)) == len(whole["count"])
    merged = {}
    for p in parts:
        merged.update(table_to_dict(p))
    assert merged == table_to_dict(whole)
    for p, t in enumerate(parts):
        assert (oracle.owner_of(t["key_hi"], t["key_lo"], 5) == p).all()


def test_tiling_closed_form():
    """Error-free reads at every start of a genome with unique canonical k-mers: the count of
    the k-mer at genome position j is #{s : s <= j <= s + L - k}, its tallies follow the same
    rule on the (k+1)-windows, and every interior k-mer is UU with the genome's neighbours."""
    rng = np.random.default_rng(21)
    G, L, k = 1500, 60, 21
    g = "".join(rng.choice(list(BASES), G))
    kmers = [g[j:j + k] for j in range(G - k + 1)]
    canon = [min(enc(w), enc("".join(COMP[c] for c in reversed(w)))) for w in kmers]
    assert len(set(canon)) == len(canon)
    reads = [(g[s:s + L], [40] * L) for s in range(G - L + 1)]
    d = table_to_dict(run_reads(reads, k, min_depth=1, ext_min=1, qcut=30))
    assert len(d) == len(kmers)
    S = G - L  # starts 0..S
    for j, w in enumerate(kmers):
        cnt = sum(1 for s in range(max(0, j + k - L), min(j, S) + 1))
        n_left = sum(1 for s in range(max(0, j + k - L), min(j - 1, S) + 1)) if j >= 1 else 0
        n_right = sum(1 for s in range(max(0, j + k + 1 - L), min(j, S) + 1)) if j + k < G else 0
        f = enc(w)
        r = enc("".join(COMP[c] for c in reversed(w)))
        tl, tr = [0] * 4, [0] * 4
        if f <= r:
            if n_left:
                tl[BASES.index(g[j - 1])] = n_left
            if n_right:
                tr[BASES.index(g[j + k])] = n_right
        else:
            if n_right:
                tl[BASES.index(COMP[g[j + k]])] = n_right
            if n_left:
                tr[BASES.index(COMP[g[j - 1]])] = n_left
        got = d[min(f, r)]
        assert got[0] == cnt and got[1] == tuple(tl) and got[2] == tuple(tr), j
        if n_left and n_right:
            assert got[3] < 4 and got[4] < 4


def test_tiny_workload_statistics():
    """Generator + oracle sanity on the tiny workload shape: the mean count of error-free genome
    k-mers is close to d (1 - (k-1)/L) (1-p)^k (the Poisson mean of the pipeline section,
    thinned by errors), and most distinct k-mers are erroneous (the k-mer analysis section
    reports over 80% for typical data)."""
    from paper_1705_11147_amd import synth
    w = synth.tiny(scale=0.25)
    r = w.reads()
    k = w.params.k
    full = oracle.run(r.ascii, r.qual, r.offsets(), k, keep_all=True, min_depth=1)
    d_keys = (full["key_hi"].astype(object) << 64) | full["key_lo"].astype(object)
    lookup = dict(zip(d_keys.tolist(), full["count"].tolist()))
    g = w.genome.tobytes().decode()
    rng = np.random.default_rng(3)
    counts = []
    for j in rng.integers(0, len(g) - k, 2000):
        s = g[j:j + k]
        key = min(enc(s), enc("".join(COMP[c] for c in reversed(s))))
        counts.append(lookup.get(key, 0))
    expected = 20 * (1 - (k - 1) / 100) * (1 - 0.01) ** k
    assert abs(np.mean(counts) - expected) < 0.6, (np.mean(counts), expected)
    erroneous = np.mean(full["count"] == 1)
    assert 0.6 < erroneous < 0.9
