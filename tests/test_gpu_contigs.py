"""Contig generation on the GPU (hm_contigs, through the C ABI) against the oracle's
(oracle.contigs).

A contig set is unique (every path and cycle of UU k-mers, spelled canonically), so the bar is
exact: the sorted list of contig strings.  Inputs come two ways: UU records the GPU exported from
its own count table (the path as a whole), and oracle tables copied in (graph shapes chosen on
purpose: circular genomes, tandem repeats, hairpins, non-UU records mixed in)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests import brute
from tests.util import pack_reads, random_read_set, read_golden

pytestmark = pytest.mark.gpu

BASES = "ACGT"


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def gpu_contigs_of_table(t, k, forward_only=False, shuffle=None):
    if shuffle is not None:  # any record order
        order = np.random.default_rng(shuffle).permutation(len(t["key_hi"]))
        t = {x: v[order] for x, v in t.items() if isinstance(v, np.ndarray)}
    r = kmer.Records.from_numpy(t, device="cuda")
    return kmer.contigs(r, k, forward_only=forward_only)


def gpu_contigs_of_reads(ascii, qual, off, k, forward_only=False, min_depth=2, read_len=None, sort=False):
    """The whole path on the GPU: count, classify, export the UU records, generate contigs."""
    dev = torch.device("cuda:0")
    a = torch.from_numpy(np.ascontiguousarray(ascii)).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(qual)).to(dev)
    if read_len:
        p = kmer.pack_reads(a, q, read_len=read_len)
    else:
        p = kmer.pack_reads(a, q, read_off=torch.from_numpy(np.ascontiguousarray(off)).to(dev))
    P = p.positions(k)
    cap = kmer.next_pow2(max(1024, 2 * P))
    kc = kmer.KmerCounter(k, cap, kmer.next_pow2(max(64, P * 10 // 64)), max(P, 1), min_depth=min_depth,
                          flags=abi.HM_FORWARD_ONLY if forward_only else 0, device=dev)
    out = kmer.Records(cap // 2, device=dev)
    kc.run([p], out, flags=abi.HM_EXPORT_UU_ONLY | (abi.HM_EXPORT_SORTED if sort else 0))
    assert kc.status() == abi.HM_OK
    return kmer.contigs(out, k, forward_only=forward_only)


def genome_reads(rng, G, L, circular=False, copies=2):
    g = "".join(rng.choice(list(BASES), G))
    src = g + g[:L] if circular else g
    starts = range(0, G if circular else G - L + 1)
    return g, [src[s:s + L] for s in starts for _ in range(copies)]


def table_of(seqs, k, **kw):
    a, q, off = pack_reads([(s, [40] * len(s)) for s in seqs])
    kw.setdefault("qcut", 0)
    return oracle.run(a, q, off, k, **kw), (a, q, off)


def test_paper_traversal_example():
    """GATCTGA (the paper's traversal example), from the GPU's own UU export."""
    g = read_golden("contig_gatctga.txt")
    k = int(g["k"][0][0])
    t, (a, q, off) = table_of(g["reads"][0], k, forward_only=True)
    assert gpu_contigs_of_reads(a, q, off, k, forward_only=True) == g["contigs"][0]
    assert gpu_contigs_of_table(t, k, forward_only=True) == g["contigs"][0]


@pytest.mark.parametrize("k", [15, 21, 31, 33, 51, 63])
@pytest.mark.parametrize("circular", [False, True])
def test_genome_one_contig_all_widths(k, circular):
    """A random genome, linear (one path: the genome less its end bases) or circular (one cycle of
    G k-mers spelled from the smallest k-mer), one- and two-word keys."""
    rng = np.random.default_rng(k + 1000 * circular)
    g, reads = genome_reads(rng, 3000, 80, circular=circular)
    t, (a, q, off) = table_of(reads, k)
    exp = oracle.contigs(t, k)
    assert len(exp) == 1
    assert gpu_contigs_of_reads(a, q, off, k) == exp
    assert gpu_contigs_of_table(t, k, shuffle=k) == exp


@pytest.mark.parametrize("k", [2, 8, 16, 21, 32, 40])
@pytest.mark.parametrize("circular", [False, True])
def test_forward_only(k, circular):
    rng = np.random.default_rng(50 + k + 1000 * circular)
    g, reads = genome_reads(rng, 1500, 60, circular=circular)
    t, (a, q, off) = table_of(reads, k, forward_only=True)
    exp = oracle.contigs(t, k, forward_only=True)
    assert gpu_contigs_of_reads(a, q, off, k, forward_only=True) == exp
    assert gpu_contigs_of_table(t, k, forward_only=True, shuffle=k) == exp


@pytest.mark.parametrize("seed,k,min_depth", [(1, 15, 2), (2, 21, 1), (3, 31, 2), (4, 33, 1), (5, 51, 2),
                                              (6, 63, 1)])
def test_error_laden_reads(seed, k, min_depth):
    """Reads with substitutions, N and lowercase: many short contigs, tips and forks."""
    ascii, qual, off = random_read_set(700 + seed, 3000, 60, 200, genome_len=20000, n_rate=0.002, lower_rate=0.01)
    t = oracle.run(ascii, qual, off, k, min_depth=min_depth, n_threads=8)
    exp = oracle.contigs(t, k)
    assert len(exp) > 50
    assert gpu_contigs_of_reads(ascii, qual, off, k, min_depth=min_depth) == exp


def test_mixed_records_and_any_order():
    """A full classified table (F and X records among the UU ones), shuffled: the non-UU records
    are not part of the graph."""
    ascii, qual, off = random_read_set(760, 2000, 80, 150, genome_len=8000)
    t = oracle.run(ascii, qual, off, 21, n_threads=8)
    assert (~oracle.uu_mask(t)).sum() > 100
    exp = oracle.contigs(t, 21)
    assert gpu_contigs_of_table(t, 21, shuffle=3) == exp


@pytest.mark.parametrize("unit", ["A", "AC", "ACGT", "ACGTTGCA", "AGCTTAGGCATCGA", "AAAAAAAAAAAAAAAAAAAAAC"])
@pytest.mark.parametrize("k", [3, 5, 9, 21])
def test_tandem_repeats_cycles_and_hairpins(unit, k):
    """Tandem repeats read on the forward strand: one-k-mer cycles (a homopolymer), palindromic
    units whose links fold back on themselves (hairpins), longer cycles."""
    g = unit * (200 // len(unit) + 3)
    for fwd in (False, True):
        t, (a, q, off) = table_of([g, g], k, forward_only=fwd)
        exp = oracle.contigs(t, k, forward_only=fwd)
        assert gpu_contigs_of_table(t, k, forward_only=fwd) == exp, (unit, k, fwd)
        assert gpu_contigs_of_reads(a, q, off, k, forward_only=fwd) == exp, (unit, k, fwd)


def test_many_cycles_and_paths():
    """Several circular genomes of different sizes and linear ones in one read set (cycles of
    lengths 1..3000 next to paths), canonical and forward-only."""
    rng = np.random.default_rng(77)
    reads = []
    for G in (40, 97, 300, 1000, 3000):
        reads += genome_reads(rng, G, 35, circular=True)[1]
        reads += genome_reads(rng, G + 100, 35)[1]
    reads += ["A" * 50] * 2 + ["ACGT" * 12] * 2
    k = 21
    for fwd in (False, True):
        t, (a, q, off) = table_of(reads, k, forward_only=fwd)
        exp = oracle.contigs(t, k, forward_only=fwd)
        assert gpu_contigs_of_reads(a, q, off, k, forward_only=fwd) == exp
        assert gpu_contigs_of_table(t, k, forward_only=fwd, shuffle=1) == exp


def test_mid_shape_whole_path():
    """The mid workload's shape at 1/200 (k=51, 150-base reads), through the GPU counting path and
    a key-ordered UU export."""
    w = synth.mid(scale=0.005)
    r = w.reads()
    k = w.params.k
    t = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=w.params.qcut, n_threads=8)
    exp = oracle.contigs(t, k)
    got = gpu_contigs_of_reads(r.ascii, r.qual, r.offsets(), k, read_len=150, sort=True)
    assert len(got) > 1000
    assert got == exp


def test_empty_and_duplicate_and_small_output():
    z = {x: np.zeros(0, np.uint64) for x in ("key_hi", "key_lo")}
    z.update(cls_l=np.zeros(0, np.uint8), cls_r=np.zeros(0, np.uint8))
    r = kmer.Records.from_numpy(z)
    cs = kmer.ContigSet(max(r.capacity, 1), 21)
    assert cs.run(r) == 0
    assert cs.to_list() == [] and int(cs.off[0].item()) == 0
    # a duplicate key: reported, no output
    rng = np.random.default_rng(8)
    g, reads = genome_reads(rng, 500, 40)
    t, _ = table_of(reads, 21)
    m = oracle.uu_mask(t)
    d = {x: np.concatenate([t[x][m], t[x][m][:1]]) for x in ("key_hi", "key_lo", "cls_l", "cls_r")}
    cs = kmer.ContigSet(len(d["key_hi"]), 21)
    st = cs.run(kmer.Records.from_numpy(d))
    assert st & abi.HM_ST_DUPLICATE and int(cs.counts[0].item()) == 0
    # outputs too small: the status says so, counts hold what is needed, run() grows them
    exp = oracle.contigs(t, 21)
    rec = kmer.Records.from_numpy(t)
    cs = kmer.ContigSet(rec.capacity, 21, seq_capacity=10, off_capacity=0)
    cs.launch(rec)
    assert int(cs.status_buf.item()) & abi.HM_ST_OUTPUT_FULL
    nc, nb = (int(x) for x in cs.counts.cpu().numpy())
    assert (nc, nb) == (len(exp), sum(len(c) for c in exp))
    assert cs.run(rec) == 0 and cs.to_list() == exp


def test_bad_arguments_rejected():
    r = kmer.Records(100)
    cs = kmer.ContigSet(100, 21)
    ex, c = r.struct(digest=False), cs.struct()
    L = abi.lib()
    import ctypes
    assert L.hm_contigs(ctypes.byref(ex), 20, 0, ctypes.byref(c), None) == abi.HM_EINVAL  # even k, canonical
    assert L.hm_contigs(ctypes.byref(ex), 64, abi.HM_FORWARD_ONLY, ctypes.byref(c), None) == abi.HM_EINVAL
    assert L.hm_contigs(ctypes.byref(ex), 21, 2, ctypes.byref(c), None) == abi.HM_EINVAL  # unknown flag
    c.work_bytes = 100
    assert L.hm_contigs(ctypes.byref(ex), 21, 0, ctypes.byref(c), None) == abi.HM_EINVAL
    c = cs.struct()
    c.work = c.work + 8
    assert L.hm_contigs(ctypes.byref(ex), 21, 0, ctypes.byref(c), None) == abi.HM_EINVAL


def test_contigs_cover_every_uu_kmer_once():
    """Every UU k-mer lies in exactly one contig, in either orientation (an invariant at any size),
    on the mid shape at 1/100."""
    w = synth.mid(scale=0.01)
    r = w.reads()
    k = w.params.k
    got = gpu_contigs_of_reads(r.ascii, r.qual, r.offsets(), k, read_len=150)
    t = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=w.params.qcut, n_threads=8)
    m = oracle.uu_mask(t)
    uu = set((int(h) << 64) | int(l) for h, l in zip(t["key_hi"][m], t["key_lo"][m]))
    seen = 0
    for c in got[:2000]:
        for i in range(len(c) - k + 1):
            x = c[i:i + k]
            assert brute.enc(min(x, brute.revcomp(x))) in uu
        seen += len(c) - k + 1
    assert sum(len(c) - k + 1 for c in got) == len(uu)


@pytest.mark.parametrize("k,fwd", [(1, False), (1, True), (3, False), (2, True)])
def test_smallest_k(k, fwd):
    """k = 1..3: a handful of keys, every link a candidate, self-loops and hairpins everywhere."""
    ascii, qual, off = random_read_set(990 + k, 300, 5, 40, genome_len=60)
    t = oracle.run(ascii, qual, off, k, min_depth=1, forward_only=fwd, n_threads=4)
    exp = oracle.contigs(t, k, forward_only=fwd)
    assert gpu_contigs_of_table(t, k, forward_only=fwd) == exp


def test_single_kmer_contigs_and_no_uu():
    """UU k-mers with no links are one-k-mer contigs (in canonical spelling); a table without UU
    records gives no contigs."""
    rng = np.random.default_rng(21)
    reads = ["".join(rng.choice(list(BASES), 23)) for _ in range(200)]  # k=21: three k-mers per read, no overlaps
    t, _ = table_of(reads * 2, 21)
    exp = oracle.contigs(t, 21)
    assert gpu_contigs_of_table(t, 21) == exp
    assert any(len(c) == 21 for c in exp)
    m = oracle.uu_mask(t)
    nouu = {x: v[~m] for x, v in t.items() if isinstance(v, np.ndarray)}
    assert len(nouu["key_hi"]) > 0
    assert gpu_contigs_of_table(nouu, 21) == [] == oracle.contigs(nouu, 21)


def test_record_count_above_capacity():
    """An export that overflowed reports more records than its buffer holds: only the buffer's
    records are read."""
    rng = np.random.default_rng(22)
    g, reads = genome_reads(rng, 800, 60)
    t, _ = table_of(reads, 21)
    r = kmer.Records.from_numpy(t)
    r.n_out.fill_(r.capacity + 12345)
    assert kmer.contigs(r, 21) == oracle.contigs(t, 21)


def test_graph_replays_match_eager():
    """hm_contigs captured in a HIP graph (its clears are fill kernels): three replays, with eager
    contig generation on another input and host synchronizations between them, each equal to the
    eager result."""
    rng = np.random.default_rng(31)
    reads = []
    for G in (60, 500, 2000):
        reads += genome_reads(rng, G, 40, circular=True)[1] + genome_reads(rng, G + 50, 40)[1]
    t, _ = table_of(reads, 21)
    exp = oracle.contigs(t, 21)
    rec = kmer.Records.from_numpy(t)
    cs = kmer.ContigSet(rec.capacity, 21)
    assert cs.run(rec) == 0 and cs.to_list() == exp  # eager; sizes the outputs
    other_t, _ = table_of(genome_reads(rng, 900, 40)[1], 21)
    other = kmer.Records.from_numpy(other_t)
    other_exp = oracle.contigs(other_t, 21)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        cs.launch(rec)  # warm-up on a side stream before capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cs.launch(rec)
    for rep in range(3):
        cs.counts.zero_()
        cs.seq.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert int(cs.status_buf.item()) == 0, rep
        assert cs.to_list() == exp, rep
        assert kmer.contigs(other, 21) == other_exp  # eager work between replays


def test_long_cycle_and_path():
    """A 300 kbp circular genome (one cycle of 3.0e5 k-mers, about 9400 rulers on it, and 6e5
    readings in the cycle jumping) beside a 300 kbp linear one, k = 31."""
    rng = np.random.default_rng(41)
    L, k = 100, 31
    reads = []
    for circ in (True, False):
        g = "".join(rng.choice(list(BASES), 300_000))
        src = g + g[:L] if circ else g
        reads += [src[s:s + L] for s in range(0, (300_000 if circ else 300_000 - L + 1), 3)]
    t, (a, q, off) = table_of(reads, k, n_threads=8)
    exp = oracle.contigs(t, k)
    lens = sorted(len(c) for c in exp)
    assert len(exp) == 2 and lens[1] == 300_000 + k - 1 and lens[0] > 299_900  # the cycle, and the path
    assert gpu_contigs_of_table(t, k, shuffle=5) == exp
    assert gpu_contigs_of_reads(a, q, off, k) == exp
