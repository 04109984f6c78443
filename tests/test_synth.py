"""Synthetic read generator: determinism and the statistics each workload recipe states."""
import numpy as np

from paper_1705_11147_amd import synth

LUT = np.zeros(256, np.uint8)
for a, b in zip(b"ACGT", b"TGCA"):
    LUT[a] = b


def truth_of(w, r):
    L = r.read_len
    idx = r.start[:, None] + np.arange(L)[None, :]
    t = w.genome[idx]
    rc = r.strand.astype(bool)
    t[rc] = LUT[t[rc][:, ::-1]]
    return t


def test_deterministic_and_batch_consistent():
    w = synth.tiny(scale=0.05)
    a = w.reads()
    b = w.reads()
    assert np.array_equal(a.ascii, b.ascii) and np.array_equal(a.qual, b.qual)
    part = w.reads(r0=100, n=50)
    assert np.array_equal(part.ascii, a.ascii[100 * 100:150 * 100])


def test_tiny_recipe_statistics():
    w = synth.tiny(scale=0.2)
    r = w.reads(keep_truth=True)
    assert r.n_reads == 40_000 and r.read_len == 100
    assert set(np.unique(r.ascii).tolist()) <= set(b"ACGT")
    err = (truth_of(w, r) != r.ascii.reshape(-1, 100)).mean()
    assert abs(err - 0.01) < 0.001
    assert abs(r.strand.mean() - 0.5) < 0.02
    q = r.qual.astype(np.int64)
    assert q.min() >= 2 and q.max() <= 41 and abs(q.mean() - 32) < 0.2
    assert abs((q >= 20).mean() - 0.98) < 0.01


def test_mid_recipe_end_bias_and_repeats():
    w = synth.mid(scale=0.01)
    r = w.reads(n=60_000, keep_truth=True)
    e = (truth_of(w, r) != r.ascii.reshape(-1, 150)).mean(axis=0)
    assert abs(e.mean() - 0.005) < 0.0007
    assert e[:5].mean() > 2.2 * e[70:80].mean()


def test_homeolog_divergence():
    arr, jobs = synth.serving_jobs(n_jobs=3, scale=0.01)
    assert np.all(np.diff(arr) >= 0)
    w = jobs[0]()
    g0 = int(w.chrom_off[1])
    a, b = w.genome[:g0], w.genome[g0:2 * g0]
    assert abs((a != b).mean() - 0.03) < 0.006
