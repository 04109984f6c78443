"""Parity at full workload size, in the launch configuration bench.py times.

The mid workload's whole table (2e9 positions, 1.0e8 kept k-mers), from the
table path and from the binned path, is compared with the oracle's record by
record (the sort-counted oracle on every host core); so are all 64 read sets of the batched workload, and one GPU's share of
the human-scale recipe at 1/10 of its reads in ten streamed batches.
Properties that hold at any size (position count, event balance,
determinism) are checked on the full tables too."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, table_digest

pytestmark = pytest.mark.gpu

THREADS = len(os.sched_getaffinity(0))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def test_mid_workload_full_size():
    w = synth.mid()
    r = w.reads()
    p = w.params
    L, k = r.read_len, p.k
    positions = r.n_reads * (L - k + 1)
    print("mid workload full size: %d reads x %d, k=%d" % (r.n_reads, L, k), flush=True)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(r.ascii).to(dev)
    q = torch.from_numpy(r.qual).to(dev)
    packed = kmer.pack_reads(a, q, read_len=L, qcut=p.qcut)
    # sizes from the cardinality pass, as bench.py does; the pass itself is checked against the
    # oracle's below
    sk = kmer.CardSketch(k, positions, device=dev)
    card = sk.run([packed], min_depth=p.min_depth)
    assert card.status == abi.HM_OK and card.positions == positions
    regs = sk.registers.cpu().numpy().view(np.uint32).copy()
    cap, bloom_words, list_cap = kmer.plan_sizes(card, n_hash=4, device=dev)
    kc = kmer.KmerCounter(k, cap, bloom_words, list_cap, n_hash=4, min_depth=p.min_depth, heavy=card, device=dev)
    out = kmer.Records(int(cap * 0.6), device=dev)
    digests = []
    for flags in (0, 0, abi.HM_EXPORT_SORTED):
        kc.run([packed], out, flags=flags)
        assert kc.status() == abi.HM_OK
        digests.append(out.digest_words())
    assert digests[0] == digests[1] == digests[2]
    st = kc.stats()
    assert st["occurrences"] == positions  # no N bases in the synthetic reads
    assert st["hit_first_lookup"] + st["bloom_tests"] + st["heavy_local"] == positions
    assert st["p2_entries"] == st["deferred"]
    got = out.to_numpy(sort=False)  # in key order: HM_EXPORT_SORTED
    del kc, out
    torch.cuda.empty_cache()
    # the binned path (the bench's timed step) on the same reads, with the bench's partition
    g, b = kmer.plan_bins(card.distinct_hi(), card.kept_hi())
    bc = kmer.BinnedCounter(k, positions, g, b, min_depth=p.min_depth, device=dev)
    bout = kmer.Records(int(len(got["count"]) * 1.2) + 4096, device=dev)
    assert bc.run(packed, bout) == 0  # no bin spills at this workload
    assert bc.status() == abi.HM_OK
    bst = bc.stats()
    assert bst["records"] == positions and bst["kept"] == len(got["count"])
    assert bout.digest_words() == digests[0]
    binned = bout.to_numpy(sort=True)
    del a, q, packed, bc, bout
    torch.cuda.empty_cache()
    hi, lo = got["key_hi"], got["key_lo"]
    assert ((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))).all()
    assert (got["count"] >= 2).all()
    assert (got["tl"].sum(1) <= got["count"]).all() and (got["tr"].sum(1) <= got["count"]).all()
    exp = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=p.qcut, min_depth=p.min_depth, n_threads=THREADS,
                     sort_count=True)
    assert exp["positions"] == positions
    assert len(exp["count"]) > 90_000_000
    assert_tables_equal(got, exp, "mid full size, every record")
    assert_tables_equal(binned, exp, "mid full size, binned path, every record")
    del exp, binned
    # the cardinality pass at full size, bit for bit
    ec = oracle.card(r.ascii, r.offsets(), k, hll_p=card.hll_p, sample_log2=card.sample_log2,
                     heavy_log2=card.heavy_log2, min_depth=p.min_depth, heavy_min=16, n_threads=THREADS)
    assert np.array_equal(regs, ec["registers"])
    assert (card.positions, card.sampled_distinct, card.sampled_kept, card.n_heavy) == (
        ec["positions"], ec["sampled_distinct"], ec["sampled_kept"], ec["n_heavy"])
    assert abs(card.estimate - ec["estimate"]) <= 1e-12 * ec["estimate"]


def test_batched_workload_every_set_full_size():
    """The batched workload at full size (64 read sets, 0.5-8 Mbp genomes at 10-60x, k=31), one
    persistent launch: every set's table equals the oracle's record by record."""
    from paper_1705_11147_amd.batch import Batch, SetSpec
    dev = torch.device("cuda:0")
    ws = synth.batched_sets(n_sets=64, scale=1.0)
    specs, host = [], []
    for w in ws:
        r = w.reads()
        d, kept = w.size_estimates()
        specs.append(SetSpec(torch.from_numpy(r.ascii).to(dev), torch.from_numpy(r.qual).to(dev), r.read_len, d,
                             kept))
        host.append(r)
    k = ws[0].params.k
    b = Batch(specs, k, device=dev)
    b.launch()
    assert b.status() == [abi.HM_OK] * len(ws)
    print("batched: %d sets, %.3g positions launched" % (len(ws), b.positions()), flush=True)
    total = 0
    for i, r in enumerate(host):
        exp = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=20, min_depth=2, n_threads=THREADS, sort_count=True)
        got = b.table(i)
        assert_tables_equal(got, exp, "batched set %d of %d" % (i, len(host)))
        total += len(exp["count"])
    assert total > 64 * 100_000


def test_human_share_ten_batches_stream():
    """One GPU's share of the human-scale recipe (interspersed repeats, owner 0 of 16) at 1/10 of its
    reads in ten batches, in bench.py's form: the cardinality pass writes the owned occurrences of
    every batch to one stream, and one pass-1 launch reads it.  The whole table equals the
    oracle's, which counts the ten batches one after another (oracle.Accumulator), and so does
    the binned path's from the same stream (hm_bin_occ, hm_count_bins)."""
    w = synth.human_share(scale=1 / 10)
    p = w.params
    dev = torch.device("cuda:0")
    nb = w.meta["batch_reads"]
    cuts = list(range(0, w.n_reads, nb)) + [w.n_reads]
    assert len(cuts) - 1 == 10
    acc = oracle.Accumulator(p.k, qcut=p.qcut, min_depth=p.min_depth, n_owners=p.n_owners, owner=p.owner,
                             sort_count=True, n_threads=THREADS)
    packs = []
    for i in range(10):
        r = w.reads(r0=cuts[i], n=cuts[i + 1] - cuts[i])
        packs.append(kmer.pack_reads(torch.from_numpy(r.ascii).to(dev), torch.from_numpy(r.qual).to(dev),
                                     read_len=r.read_len, qcut=p.qcut))
        acc.add(r.ascii, r.qual, r.offsets())
        del r
    sk = kmer.CardSketch(p.k, w.positions, n_owners=p.n_owners, owner=p.owner, device=dev)
    occ = kmer.OccStream.for_windows(w.positions, p.n_owners, len(packs), device=dev)
    card = sk.run(packs, min_depth=p.min_depth, occ=occ)
    assert card.status == abi.HM_OK and not occ.overflowed()
    cap, bw, lcap = kmer.plan_sizes(card, device=dev)
    kc = kmer.KmerCounter(p.k, cap, bw, lcap, n_owners=p.n_owners, owner=p.owner, heavy=card, device=dev)
    out = kmer.Records(int(min(kc.capacity, card.kept_hi() * 1.3 + 1024)), device=dev)
    kc.run_occ(occ, out, flags=abi.HM_EXPORT_SORTED, fused=True)
    assert kc.status() == abi.HM_OK
    assert kc.stats()["occurrences"] == card.positions
    got = out.to_numpy(sort=False)  # key order
    exp = acc.finish()
    assert exp["positions"] == w.positions
    assert len(exp["count"]) > 5_000_000
    assert_tables_equal(got, exp, "human share 1/10, ten batches through the stream")
    # the same stream through the binned path (hm_bin_occ, hm_count_bins), as bench.py times it
    n_tab = len(got["count"])
    del kc, out, got
    torch.cuda.empty_cache()
    g, b = kmer.plan_bins(card.distinct_hi(), card.kept_hi(), False)
    bc = kmer.BinnedCounter(p.k, occ.capacity, g, b, min_depth=p.min_depth, n_owners=p.n_owners, owner=p.owner,
                            device=dev)
    bout = kmer.Records(int(n_tab * 1.2) + 4096, device=dev)
    bc.bin_occ(occ)
    bc.count(bout)
    bc.finish(bout)
    abi.check(bc.status(), "binned share 1/10")
    st = bc.stats()
    assert st["records"] == card.positions
    print("binned: 2^%d bins, %d spilled bins" % (g + b, st["spilled_bins"]), flush=True)
    assert_tables_equal(bout.to_numpy(sort=True), exp, "human share 1/10, the stream through the binned path")


def test_human_share_streamed_batches():
    """The human-scale share's recipe (interspersed repeats, owner 0 of 16) at 1/200 scale, with its
    reads streamed through pass 1 in four batches into one table."""
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
    # one cardinality sketch over the four batches sizes the owner's table
    sk = kmer.CardSketch(p.k, w.positions, n_owners=p.n_owners, owner=p.owner, device=dev)
    card = sk.run(packs, min_depth=p.min_depth)
    assert card.status == abi.HM_OK
    cap, bw, lcap = kmer.plan_sizes(card, pass1_launches=4, device=dev)
    kc = kmer.KmerCounter(p.k, cap, bw, lcap, n_owners=p.n_owners, owner=p.owner, device=dev)
    kc.reset()
    for pk in packs:
        kc.insert(pk)
    torch.cuda.synchronize()
    del packs
    kc.count()
    kc.classify()
    out = kmer.Records(kc.capacity)
    kc.export(out)
    assert kc.status() == abi.HM_OK
    got = out.to_numpy()
    ascii = np.concatenate([r.ascii for r in host])
    qual = np.concatenate([r.qual for r in host])
    off = np.arange(n + 1, dtype=np.int64) * w.read_len
    exp = oracle.run(ascii, qual, off, p.k, qcut=p.qcut, n_owners=p.n_owners, owner=p.owner, n_threads=THREADS,
                     split_reads=True)
    assert_tables_equal(got, exp, "human share 1/200")
    assert out.digest_words() == table_digest(exp)
    assert (oracle.owner_of(got["key_hi"], got["key_lo"], 16) == 0).all()


def _codes(t):
    lut = torch.full((256,), 255, dtype=torch.uint8, device=t.device)
    for i, b in enumerate(b"ACGT"):
        lut[b] = i
    return lut[t.long()]


def _window_keys(c, k, valid):
    """Canonical (hi, lo) words of every window start p with valid[p] (2-bit codes c, first base most
    significant), computed with torch on the device: a checker, independent of the HIP path."""
    n = c.numel() - k + 1
    p = torch.nonzero(valid[:n]).flatten()
    lo_bases = min(k, 32)
    hi_bases = k - lo_bases

    def words(base_at):
        hi = torch.zeros(p.numel(), dtype=torch.int64, device=c.device)
        lo = torch.zeros_like(hi)
        for j in range(hi_bases):
            hi = (hi << 2) | base_at(j)
        for j in range(hi_bases, k):
            lo = (lo << 2) | base_at(j)
        return hi, lo

    fh, fl = words(lambda j: c[p + j].long())
    rh, rl = words(lambda j: 3 - c[p + k - 1 - j].long())
    s = -2 ** 63  # flip the sign bit: signed order of the flipped words = unsigned order
    rc_less = (rh < fh) | ((rh == fh) & ((rl ^ s) < (fl ^ s)))
    return torch.where(rc_less, rh, fh), torch.where(rc_less, rl, fl)


def test_mid_workload_contigs_full_size():
    """Contig generation at full size (the mid workload's 1.0e8 UU k-mers, the configuration bench.py
    times), checked by properties that hold at any size: the contigs' windows are exactly the UU
    k-mers, each once (device-side, with torch); and on 300 sampled contigs, consecutive k-mers are
    linked from both ends, the ends do not extend, and the spelling is canonical."""
    w = synth.mid()
    r = w.reads()
    p = w.params
    L, k = r.read_len, p.k
    positions = r.n_reads * (L - k + 1)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(r.ascii).to(dev)
    q = torch.from_numpy(r.qual).to(dev)
    packed = kmer.pack_reads(a, q, read_len=L, qcut=p.qcut)
    del a, q
    card = kmer.CardSketch(k, positions, device=dev).run([packed], min_depth=p.min_depth)
    cap, bw, lcap = kmer.plan_sizes(card, n_hash=4, device=dev)
    kc = kmer.KmerCounter(k, cap, bw, lcap, n_hash=4, min_depth=p.min_depth, heavy=card, device=dev)
    uu = kmer.Records(int(cap * 0.5), device=dev)
    kc.run([packed], uu, flags=abi.HM_EXPORT_UU_ONLY, fused=True)
    assert kc.status() == abi.HM_OK
    del kc, packed
    torch.cuda.empty_cache()
    n_uu = int(uu.n_out.item())
    print("mid full size: %d UU k-mers" % n_uu, flush=True)
    cs = kmer.ContigSet(uu.capacity, k, device=dev)
    assert cs.run(uu) == 0
    nc, nb = (int(x) for x in cs.counts.cpu().numpy())
    assert nb - nc * (k - 1) == n_uu and nc > 100_000
    off = cs.off[:nc + 1]
    assert (off[1:] - off[:-1] >= k).all() and int(off[0].item()) == 0 and int(off[-1].item()) == nb
    seq = cs.seq[:nb]
    c = _codes(seq)
    assert (c < 4).all()
    # windows inside a contig: p + k <= end of p's contig
    cid = torch.bucketize(torch.arange(nb, device=dev), off[1:], right=True)
    valid = torch.arange(nb, device=dev) + k <= off[1:][cid]
    wh, wl = _window_keys(c, k, valid)
    assert wh.numel() == n_uu
    got = torch.unique(torch.stack([wh, wl], 1), dim=0)
    exp = torch.unique(torch.stack([uu.key_hi[:n_uu], uu.key_lo[:n_uu]], 1), dim=0)
    assert got.shape == exp.shape and torch.equal(got, exp), "contig windows differ from the UU k-mers"
    del got, exp, wh, wl, cid, valid, c
    # sampled contigs, with Python strings, against the export's keys and classes
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(nc, 300, replace=False))
    offs = off.cpu().numpy()
    sb = seq.cpu().numpy().tobytes()
    contigs = [sb[offs[i]:offs[i + 1]].decode() for i in pick]
    his = uu.key_hi[:n_uu].cpu().numpy().view(np.uint64)
    from tests import brute

    def canon(x):
        return min(x, brute.revcomp(x))

    want = set()
    for ctg in contigs:
        for i in range(len(ctg) - k + 1):
            want.add(brute.enc(canon(ctg[i:i + k])) >> 64)
        for x in ("ACGT"):
            want.add(brute.enc(canon(x + ctg[:k - 1])) >> 64)
            want.add(brute.enc(canon(ctg[-(k - 1):] + x)) >> 64)
    m = np.isin(his, np.array(sorted(want), dtype=np.uint64))
    los = uu.key_lo[:n_uu].cpu().numpy().view(np.uint64)[m]
    cls_l = uu.cls_l[:n_uu].cpu().numpy()[m]
    cls_r = uu.cls_r[:n_uu].cpu().numpy()[m]
    table = {(int(h) << 64) | int(l): (int(a_), int(b_)) for h, l, a_, b_ in zip(his[m], los, cls_l, cls_r)}
    B = "ACGT"

    def ext(s):  # (left, right) extension of the oriented k-mer s, or None if not a UU k-mer
        cs_ = canon(s)
        v = table.get(brute.enc(cs_))
        if v is None:
            return None
        l_, r_ = B[v[0]], B[v[1]]
        return (l_, r_) if cs_ == s else (brute.COMP[r_], brute.COMP[l_])

    def linked_right(s):  # the k-mer s links to on its right (both ends agree, no hairpin), or None
        e = ext(s)
        t = s[1:] + e[1]
        et = ext(t)
        if et is None or et[0] != s[0] or (canon(t) == canon(s) and t != s):
            return None
        return t

    cycles = 0
    for ctg in contigs:
        ks = [ctg[i:i + k] for i in range(len(ctg) - k + 1)]
        for x, y in zip(ks, ks[1:]):
            assert linked_right(x) == y, ctg[:60]
        nxt = linked_right(ks[-1])
        prv = linked_right(brute.revcomp(ks[0]))  # the left link of the first k-mer, read backwards
        if nxt is not None:  # a cycle: it closes on its first k-mer and starts at its smallest key
            cycles += 1
            assert nxt == ks[0] and prv == brute.revcomp(ks[-1])
            assert ks[0] == canon(ks[0]) and brute.enc(ks[0]) == min(brute.enc(canon(x)) for x in ks)
        else:
            assert prv is None
            assert ctg <= brute.revcomp(ctg)
    print("sampled 300 contigs (%d cycles): links, ends and orientation hold" % cycles)
