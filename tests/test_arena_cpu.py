"""Device arena bookkeeping on the CPU (the arena over a host tensor): placement against a
byte-map model, hole merging, slabs, and the slab sizes the serving backend reserves for each
structure, checked against the bytes the constructors actually take."""
import os

import numpy as np
import pytest
import torch

from paper_1705_11147_amd import abi
from paper_1705_11147_amd.arena import ALIGN, DeviceArena, Slab, aligned


def check_model(a: DeviceArena, owner: np.ndarray):
    """The arena's holes are exactly the free runs of the byte map, merged and sorted."""
    runs, i, n = [], 0, len(owner)
    while i < n:
        if owner[i] == 0:
            j = i
            while j < n and owner[j] == 0:
                j += 1
            runs.append((i * ALIGN, (j - i) * ALIGN))
            i = j
        else:
            i += 1
    assert a.holes() == runs
    assert a.used == int((owner != 0).sum()) * ALIGN


def test_best_fit_placement_and_merging():
    rng = np.random.default_rng(5)
    units = 512
    a = DeviceArena(units * ALIGN, device="cpu")
    owner = np.zeros(units, np.int32)
    live = {}
    tag = 0
    for step in range(3000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            off = list(live)[int(rng.integers(len(live)))]
            a.release(off)
            owner[off // ALIGN: off // ALIGN + live.pop(off)] = 0
        else:
            n = int(rng.integers(1, 40))
            high = bool(rng.integers(2))
            holes = a.holes()
            fits = [h for h in holes if h[1] >= n * ALIGN]
            assert a.fits([n * ALIGN]) == bool(fits)
            off = a.alloc(n * ALIGN - int(rng.integers(ALIGN)), high=high)  # any size rounds up
            if not fits:
                assert off is None
                continue
            best = min(fits, key=lambda h: h[1])[1]  # the smallest hole that fits
            hole = [h for h in fits if h[1] == best]
            assert any(off == (h[0] + h[1] - n * ALIGN if high else h[0]) for h in hole)
            assert (owner[off // ALIGN: off // ALIGN + n] == 0).all()
            tag += 1
            owner[off // ALIGN: off // ALIGN + n] = tag
            live[off] = n
        check_model(a, owner)
    for off in list(live):
        a.release(off)
    assert a.holes() == [(0, units * ALIGN)] and a.used == 0


def test_fits_simulates_several_blocks():
    a = DeviceArena(100 * ALIGN, device="cpu")
    x = a.alloc(30 * ALIGN)
    a.alloc(10 * ALIGN)
    a.release(x)  # holes: 30 and 60 units
    assert a.fits([30 * ALIGN, 60 * ALIGN])
    assert a.fits([60 * ALIGN, 30 * ALIGN])
    assert not a.fits([40 * ALIGN, 40 * ALIGN])
    assert not a.fits([61 * ALIGN])
    assert a.largest_hole() == 60 * ALIGN


def test_slab_pieces_views_and_spill():
    a = DeviceArena(64 * ALIGN, device="cpu")
    s = Slab(a, 4 * ALIGN)
    x = s.empty(10, torch.int64)
    y = s.zeros(3, torch.int32)
    assert x.numel() == 10 and x.dtype == torch.int64 and y.tolist() == [0, 0, 0]
    assert (y.data_ptr() - x.data_ptr()) == ALIGN  # each piece 256-byte aligned
    x.fill_(7)
    assert y.tolist() == [0, 0, 0]
    assert a.spills == 0
    z = s.empty(3 * ALIGN // 8, torch.int64)  # does not fit the 2 units left: a block of its own
    assert a.spills == 1 and z.numel() == 3 * ALIGN // 8
    assert a.used == 4 * ALIGN + 3 * ALIGN
    s.release()
    s.release()  # idempotent
    assert a.used == 0
    with pytest.raises(MemoryError):
        Slab(a, 65 * ALIGN)
    with pytest.raises(RuntimeError):
        s.empty(1, torch.uint8)
    assert aligned(1) == ALIGN and aligned(ALIGN) == ALIGN and aligned(ALIGN + 1) == 2 * ALIGN


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(abi._build.SO):
        pytest.skip("libhm_kmer.so not built")
    return abi.lib()


def used_by(build):
    """Bytes a constructor takes from a slab (CPU tensors), and that it spilled nothing."""
    a = DeviceArena(1 << 28, device="cpu")
    s = Slab(a, 1 << 27)
    build(s)
    assert a.spills == 0
    return s.cursor


@pytest.mark.parametrize("cap,bw,lcap,heavy,min_depth,present", [
    (1 << 10, 64, 1000, 0, 2, True), (1 << 12, 1 << 12, 5000, 3, 2, True), (3000, 100, 1, 0, 1, True),
    (1 << 14, 1 << 10, 123457, 17, 2, False), (5000, 1 << 13, 77, 0, 3, True)])
def test_counter_bytes_match_the_constructor(L, cap, bw, lcap, heavy, min_depth, present):
    from paper_1705_11147_amd.kmer import KmerCounter
    hk = np.arange(2 * heavy, dtype=np.uint64).reshape(-1, 2) if heavy else None
    got = used_by(lambda s: KmerCounter(31, cap, bw, lcap, min_depth=min_depth, heavy=hk, present_filter=present,
                                        device="cpu", alloc=s))
    assert got == KmerCounter.bytes_for(cap, bw, lcap, heavy, min_depth=min_depth, present_filter=present)


@pytest.mark.parametrize("n", [0, 1, 1000, 123457])
def test_records_bytes_match_the_constructor(n):
    from paper_1705_11147_amd.kmer import Records
    assert used_by(lambda s: Records(n, device="cpu", alloc=s)) == Records.bytes_for(n)


@pytest.mark.parametrize("hint", [1, 5000, 1 << 20, 3 * 10 ** 7])
def test_sketch_bytes_match_the_constructor(L, hint):
    from paper_1705_11147_amd.kmer import CardSketch
    assert used_by(lambda s: CardSketch(31, hint, device="cpu", alloc=s)) == CardSketch.bytes_for(hint)


@pytest.mark.parametrize("n_bases", [0, 1, 63, 64, 150 * 1000 + 7])
def test_packed_bytes_match(L, n_bases):
    from paper_1705_11147_amd.kmer import new_packed, packed_bytes
    assert used_by(lambda s: new_packed(n_bases, "cpu", s)) == packed_bytes(n_bases)
