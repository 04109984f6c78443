"""hm_export_table_static, the entry point for callers that cannot allocate:
a key-ordered export whose scratch is the library's own device array.  Its
output must equal hm_export_table's with a caller-owned scratch, record by
record (integer output: tolerance 0), on consecutive calls that reuse the
array with a smaller input the second time; a capacity past the array's
limit is refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1705_11147_amd import abi, kmer
from tests.util import random_read_set

pytestmark = pytest.mark.gpu

FIELDS = ("key_hi", "key_lo", "count", "tl", "tr", "cls_l", "cls_r")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    torch.cuda.set_device(0)


def counted(seed, k, n_reads):
    """A counted table of random reads, and a record capacity that fits its export."""
    ascii, qual, off = random_read_set(seed, n_reads, 80, 160, genome_len=60000)
    dev = torch.device("cuda:0")
    packed = kmer.pack_reads(torch.from_numpy(ascii).to(dev), torch.from_numpy(qual).to(dev),
                             read_off=torch.from_numpy(off).to(dev), qcut=20)
    P = packed.positions(k)
    kc = kmer.KmerCounter(k, kmer.next_pow2(2 * P), kmer.next_pow2(max(64, P // 4)), P + kmer.list_slack(),
                          device=dev)
    kc.reset()
    kc.insert(packed)
    kc.count()
    torch.cuda.synchronize()
    assert kc.status() == abi.HM_OK
    return kc


def exports(kc, capacity, flags):
    """(caller-scratch export, static-scratch export) of the same table, in key order."""
    a = kmer.Records(capacity)
    b = kmer.Records(capacity)
    kc.export(a, flags | abi.HM_EXPORT_SORTED)
    kc.export(b, flags | abi.HM_EXPORT_SORTED, static=True)
    assert kc.status() == abi.HM_OK
    return a, b


def assert_same(a, b, what):
    na, nb = int(a.n_out.item()), int(b.n_out.item())
    assert na == nb > 0, (what, na, nb)
    x, y = a.to_numpy(sort=False), b.to_numpy(sort=False)  # device order: both key-ordered
    for f in FIELDS:
        assert np.array_equal(x[f], y[f]), "%s: field %s differs" % (what, f)
    assert a.digest_words() == b.digest_words()
    hi, lo = x["key_hi"], x["key_lo"]
    assert ((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))).all(), what


@pytest.mark.parametrize("k", [21, 51])
def test_static_scratch_equals_caller_scratch_twice(k):
    """Two calls in a row on the shared array, the second with a smaller table."""
    big = counted(1000 + k, k, 3000)
    a, b = exports(big, abi.HM_EXPORT_STATIC_MAX_RECORDS, abi.HM_EXPORT_CLASSIFY)
    assert_same(a, b, "first call, k=%d" % k)
    n_big = int(a.n_out.item())
    small = counted(2000 + k, k, 400)
    a, b = exports(small, abi.HM_EXPORT_STATIC_MAX_RECORDS // 4, abi.HM_EXPORT_CLASSIFY | abi.HM_EXPORT_ALL)
    assert_same(a, b, "second call (smaller), k=%d" % k)
    assert int(a.n_out.item()) < n_big


def test_static_scratch_limit_and_unsorted():
    kc = counted(7, 31, 300)
    too_big = kmer.Records(abi.HM_EXPORT_STATIC_MAX_RECORDS + 1)
    e = too_big.struct(True, 2, 2)
    rc = abi.lib().hm_export_table_static(ctypes.byref(kc.table), abi.HM_EXPORT_SORTED | abi.HM_EXPORT_CLASSIFY,
                                          ctypes.byref(e), None)
    assert rc == abi.HM_EINVAL and "static scratch" in abi.last_error()
    # without HM_EXPORT_SORTED no scratch is needed: any capacity, same records as the plain export
    a, b = kmer.Records(1 << 20), kmer.Records(1 << 20)
    kc.export(a, abi.HM_EXPORT_CLASSIFY)
    kc.export(b, abi.HM_EXPORT_CLASSIFY, static=True)
    assert int(a.n_out.item()) == int(b.n_out.item()) > 0
    assert a.digest_words() == b.digest_words()
