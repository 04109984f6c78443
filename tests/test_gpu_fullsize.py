"""Parity at full workload size, in the launch configuration bench.py times.

The whole table of the mid workload (2e9 positions) is too large for the CPU
oracle to rebuild within a test, so the oracle computes one key shard
(1/64 of the keys, selected by a hash independent of the table layout) from
all reads, and the GPU's full export is cut to the same shard and compared
record by record.  Properties that hold at any size (position count, event
balance, determinism) are checked on the full table."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1705_11147_amd import abi, kmer, synth
from tests.util import assert_tables_equal, table_digest

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def shard(t, n, s):
    m = oracle.shard_of(t["key_hi"], t["key_lo"], n) == s
    return {x: v[m] for x, v in t.items() if isinstance(v, np.ndarray)}


def test_mid_workload_full_size_sampled():
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
    del a, q, packed, kc, out
    torch.cuda.empty_cache()
    hi, lo = got["key_hi"], got["key_lo"]
    assert ((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))).all()
    assert (got["count"] >= 2).all()
    assert (got["tl"].sum(1) <= got["count"]).all() and (got["tr"].sum(1) <= got["count"]).all()
    n_shards, s = 64, 5
    g = shard(got, n_shards, s)  # a filter keeps the key order
    exp = oracle.run(r.ascii, r.qual, r.offsets(), k, qcut=p.qcut, min_depth=p.min_depth, n_shards=n_shards,
                     shard=s, n_threads=THREADS, split_reads=True)
    assert exp["positions"] == positions
    assert len(exp["count"]) > 1_000_000
    assert_tables_equal(g, exp, "mid full size, shard %d/%d" % (s, n_shards))
    # the cardinality pass at full size, bit for bit
    ec = oracle.card(r.ascii, r.offsets(), k, hll_p=card.hll_p, sample_log2=card.sample_log2,
                     heavy_log2=card.heavy_log2, min_depth=p.min_depth, heavy_min=16, n_threads=THREADS)
    assert np.array_equal(regs, ec["registers"])
    assert (card.positions, card.sampled_distinct, card.sampled_kept, card.n_heavy) == (
        ec["positions"], ec["sampled_distinct"], ec["sampled_kept"], ec["n_heavy"])
    assert abs(card.estimate - ec["estimate"]) <= 1e-12 * ec["estimate"]


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
