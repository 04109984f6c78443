"""Pins of the oracle's contig generation (section "Parallel contig generation": UU k-mers in a
de Bruijn table, subcontigs grown by lookups until a lookup fails, connected components are the
contigs).  References: the paper's traversal example (tests/golden), a Python brute force over
strings (tests/brute.contigs), closed forms (a tiled linear or circular genome) and invariants."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests import brute
from tests.util import pack_reads, read_golden

BASES = "ACGT"


def table_of(seqs, k, **kw):
    a, q, off = pack_reads([(s, [40] * len(s)) for s in seqs])
    kw.setdefault("qcut", 0)
    return oracle.run(a, q, off, k, **kw)


def test_paper_traversal_example():
    """GATCTGA: the component explored from the seed CTG."""
    g = read_golden("contig_gatctga.txt")
    k = int(g["k"][0][0])
    t = table_of(g["reads"][0], k, forward_only=True)
    uu = oracle.uu_mask(t)
    assert sorted(int(x) for x in t["key_lo"][uu]) == sorted(brute.enc(w) for w in g["uu"][0])
    assert oracle.contigs(t, k, forward_only=True) == g["contigs"][0]


def genome_reads(rng, G, L, circular=False):
    g = "".join(rng.choice(list(BASES), G))
    src = g + g[:L] if circular else g
    starts = range(0, G if circular else G - L + 1)
    return g, [src[s:s + L] for s in starts for _ in range(2)]


@pytest.mark.parametrize("k", [15, 21, 31])
def test_linear_genome_is_one_contig(k):
    """Error-free reads at every start of a random genome whose k-mers are unique: one contig, the
    genome without its first and last base (the end k-mers lack an extension)."""
    rng = np.random.default_rng(k)
    g, reads = genome_reads(rng, 3000, 60)
    got = oracle.contigs(table_of(reads, k), k)
    inner = g[1:-1]
    assert got == [min(inner, brute.revcomp(inner))]


@pytest.mark.parametrize("k", [15, 21])
def test_circular_genome_is_one_cycle(k):
    """Reads of a circular genome: every k-mer is UU and the k-mers form one cycle of G nodes,
    spelled from the smallest k-mer in its key orientation."""
    rng = np.random.default_rng(100 + k)
    g, reads = genome_reads(rng, 2000, 50, circular=True)
    got = oracle.contigs(table_of(reads, k), k)
    assert len(got) == 1 and len(got[0]) == 2000 + k - 1
    c = got[0]
    assert c[:k] == min(min(w, brute.revcomp(w)) for w in ((g + g)[i:i + k] for i in range(2000)))
    ring = g + g
    assert c[:2000] in ring or brute.revcomp(c)[-2000:] in ring


read_st = st.text(alphabet="ACGT", min_size=5, max_size=40)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seqs=st.lists(read_st, min_size=1, max_size=8), k=st.sampled_from([3, 5, 7]), fwd=st.booleans())
def test_contigs_equal_brute_force(seqs, k, fwd):
    reads = seqs + seqs  # depth 2: the reads' interior k-mers pass the filter
    t = table_of(reads, k, forward_only=fwd)
    bt = brute.brute([(s, [40] * len(s)) for s in reads], k, qcut=0, forward_only=fwd)
    assert oracle.contigs(t, k, forward_only=fwd) == brute.contigs(bt, k, forward_only=fwd)


@pytest.mark.parametrize("motif,k", [("TTAGGG", 7), ("AC", 5), ("AATGG", 9), ("ACGT", 5)])
def test_tandem_repeats_and_palindromes(motif, k):
    """Tandem repeats give cycles and palindromic k-mer neighbourhoods (ACGT is its own reverse
    complement): the oracle agrees with the brute force."""
    rng = np.random.default_rng(len(motif) * k)
    arr = motif * 30
    flank = "".join(rng.choice(list(BASES), 40))
    reads = [flank + arr + flank[::-1], arr, arr[3:] + flank] * 2
    for fwd in (False, True):
        t = table_of(reads, k, forward_only=fwd)
        bt = brute.brute([(s, [40] * len(s)) for s in reads], k, qcut=0, forward_only=fwd)
        assert oracle.contigs(t, k, forward_only=fwd) == brute.contigs(bt, k, forward_only=fwd)


def test_every_uu_kmer_in_exactly_one_contig_and_rc_invariance():
    rng = np.random.default_rng(7)
    g = "".join(rng.choice(list(BASES), 5000))
    reads = []
    for _ in range(600):
        s = int(rng.integers(0, 4900))
        r = list(g[s:s + 100])
        for j in range(100):
            if rng.random() < 0.005:
                r[j] = BASES[(BASES.index(r[j]) + 1) % 4]
        reads.append("".join(r))
    k = 15
    t = table_of(reads, k)
    got = oracle.contigs(t, k)
    uu = {(int(h) << 64) | int(l) for h, l in zip(t["key_hi"][oracle.uu_mask(t)], t["key_lo"][oracle.uu_mask(t)])}
    seen = []
    for c in got:
        for i in range(len(c) - k + 1):
            w = c[i:i + k]
            seen.append(brute.enc(min(w, brute.revcomp(w))))
    assert sorted(seen) == sorted(uu)
    assert oracle.contigs(table_of([brute.revcomp(r) for r in reads], k), k) == got


def test_one_sided_extension_is_not_a_link():
    """x = ACGTA has right extension C, which spells y = CGTAC; but the A before y is low quality
    where x precedes it, and y's unique left extension is G (from other reads).  The extension
    does not agree from both ends, so x and y are separate contigs (worked by hand, k = 5,
    forward strand, Q20)."""
    reads = [("ACGTAC", [0, 40, 40, 40, 40, 40]), ("GCGTACT", [40] * 7), ("TACGTAC", [40, 0, 40, 40, 40, 40, 40])]
    reads = reads + reads
    a, q, off = pack_reads(reads)
    t = oracle.run(a, q, off, 5, forward_only=True, qcut=20)
    d = {int(l): (int(cl), int(cr)) for l, cl, cr in zip(t["key_lo"], t["cls_l"], t["cls_r"])}
    assert d[brute.enc("ACGTA")] == (BASES.index("T"), BASES.index("C"))
    assert d[brute.enc("CGTAC")] == (BASES.index("G"), BASES.index("T"))
    got = oracle.contigs(t, 5, forward_only=True)
    assert "ACGTA" in got and "CGTAC" in got and not any("ACGTAC" in c for c in got)
    bt = brute.brute(reads, 5, qcut=20, forward_only=True)
    assert got == brute.contigs(bt, 5, forward_only=True)
    for fwd in (True, False):  # the same reads with canonical keys, against the brute force
        t = oracle.run(a, q, off, 5, forward_only=fwd, qcut=20)
        assert oracle.contigs(t, 5, forward_only=fwd) == brute.contigs(brute.brute(reads, 5, qcut=20,
                                                                                   forward_only=fwd), 5,
                                                                       forward_only=fwd)
