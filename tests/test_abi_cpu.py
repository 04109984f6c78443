"""C ABI checks that need no GPU: the library loads, exports every function
include/hm_kmer.h declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

from paper_1705_11147_amd import abi

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(INCLUDE, h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names.update(re.findall(r"^[a-z_][a-z0-9_ \*]*?\b(hm_[a-z0-9_]+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(abi._build.SO):
        pytest.skip("libhm_kmer.so not built")
    return abi.lib()


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("hm_pack_reads", "hm_bloom_insert", "hm_kmer_count", "hm_classify_ext", "hm_export_table"):
        assert n in names
    assert set(names) == set(abi.SIGNATURES), set(names) ^ set(abi.SIGNATURES)


def test_every_declared_symbol_is_exported(L):
    for n in declared_functions():
        assert hasattr(L, n), n


def test_sizes(L):
    assert L.hm_abi_version() == 2
    assert L.hm_table_bytes(1 << 20) == 64 << 20
    assert L.hm_bloom_bytes(1024) == 8192
    assert L.hm_mask_words(0) == 3 and L.hm_mask_words(64) == 4 and L.hm_mask_words(130) == 5
    assert L.hm_bases2_words(130) == 10
    assert L.hm_list_bytes(10) == 170


def P(**kw):
    d = dict(k=21, min_depth=2, ext_min=2, n_owners=1, owner=0, flags=0, seed=1)
    d.update(kw)
    return abi.Params(**d)


@pytest.mark.parametrize("bad", [dict(k=0), dict(k=64), dict(k=20), dict(min_depth=0), dict(ext_min=0),
                                 dict(n_owners=0), dict(n_owners=4, owner=4), dict(flags=64)])
def test_check_params_rejects(L, bad):
    assert L.hm_check_params(ctypes.byref(P(**bad))) == abi.HM_EINVAL
    assert abi.last_error()


@pytest.mark.parametrize("good", [dict(), dict(k=1), dict(k=63), dict(k=20, flags=abi.HM_FORWARD_ONLY),
                                  dict(n_owners=16, owner=15), dict(flags=abi.HM_BLOOM_BYPASS | abi.HM_CHECKED),
                                  dict(flags=abi.HM_BLOOM_IN_TABLE | abi.HM_CHECKED)])
def test_check_params_accepts(L, good):
    assert L.hm_check_params(ctypes.byref(P(**good))) == abi.HM_OK


def test_host_side_rejections_touch_no_device(L):
    # each of these fails argument validation before any HIP call
    assert L.hm_pack_reads(None, None, -1, 0, 20, None, None, None, None) == abi.HM_EINVAL
    assert L.hm_pack_reads(None, None, 10, 0, 20, 8, 8, 8, None) == abi.HM_EINVAL
    t = abi.Table(64, 1000, 0, 21, 64, None)  # capacity not a power of two
    assert L.hm_table_init(ctypes.byref(t), None) == abi.HM_EINVAL
    t = abi.Table(65, 1024, 0, 21, 64, None)  # misaligned slots
    assert L.hm_table_init(ctypes.byref(t), None) == abi.HM_EINVAL
    b = abi.Bloom(64, 1000, 4)
    assert L.hm_bloom_init(ctypes.byref(b), 0, None) == abi.HM_EINVAL
    b = abi.Bloom(64, 1024, 9)
    assert L.hm_bloom_init(ctypes.byref(b), 0, None) == abi.HM_EINVAL
    assert L.hm_list_init(None, None) == abi.HM_EINVAL
    t = abi.Table(64, 1024, 0, 31, 64, None)
    r = abi.Reads(8, 8, 8, None, 10, 100, 0)  # read_len 0 without offsets
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_BYPASS)), None,
                             ctypes.byref(t), None, None) == abi.HM_EINVAL
    r = abi.Reads(8, 8, 8, None, 10, 100, 150)  # 10 reads of 150 > 100 bases
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_BYPASS)), None,
                             ctypes.byref(t), None, None) == abi.HM_EINVAL
    r = abi.Reads(8, 8, 8, None, 1, 100, 100)
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=21)), None, ctypes.byref(t), None,
                             None) == abi.HM_EINVAL  # k mismatch with the table
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31)), None, ctypes.byref(t), None,
                             None) == abi.HM_EINVAL  # Bloom needed
    # the filter in the table still needs n_hash from hm_bloom_t (its words are not used)
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_IN_TABLE)), None,
                             ctypes.byref(t), None, None) == abi.HM_EINVAL
    b = abi.Bloom(None, 0, 0)
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_IN_TABLE)), ctypes.byref(b),
                             ctypes.byref(t), None, None) == abi.HM_EINVAL
    assert "n_hash" in abi.last_error()
    b = abi.Bloom(None, 0, 4)  # accepted: the next check is the list's
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_IN_TABLE)), ctypes.byref(b),
                             ctypes.byref(t), None, None) == abi.HM_EINVAL
    assert "list" in abi.last_error()
    e = abi.Export(None, None, None, None, None, None, None, 10, 64, None)
    assert L.hm_export_table(ctypes.byref(t), 0, ctypes.byref(e), None) == abi.HM_EINVAL
    assert L.hm_export_table(ctypes.byref(t), 99, ctypes.byref(e), None) == abi.HM_EINVAL


def test_occ_stream_rejections(L):
    """The owned-occurrence stream's entry points reject bad arguments on the host."""
    assert L.hm_occ_bytes(10) == 170
    assert L.hm_occ_init(None, None) == abi.HM_EINVAL
    o = abi.Occ(64, 64, 10, None)  # no counter
    assert L.hm_occ_init(ctypes.byref(o), None) == abi.HM_EINVAL
    o = abi.Occ(None, None, 10, 64)  # arrays missing for a non-empty stream
    assert L.hm_occ_init(ctypes.byref(o), None) == abi.HM_EINVAL
    o = abi.Occ(72, 64, 10, 64)  # keys not 16-byte aligned
    assert L.hm_occ_init(ctypes.byref(o), None) == abi.HM_EINVAL
    assert "aligned" in abi.last_error()
    t = abi.Table(64, 1024, 0, 31, 64, None)
    good = abi.Occ(64, 64, 10, 64)
    # pass 1 over a stream: the same parameter, table, filter and list checks as over reads
    assert L.hm_bloom_insert_occ(ctypes.byref(o), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_BYPASS)), None,
                                 ctypes.byref(t), None, None) == abi.HM_EINVAL
    assert L.hm_bloom_insert_occ(ctypes.byref(good), ctypes.byref(P(k=21, flags=abi.HM_BLOOM_BYPASS)), None,
                                 ctypes.byref(t), None, None) == abi.HM_EINVAL  # k mismatch with the table
    assert L.hm_bloom_insert_occ(ctypes.byref(good), ctypes.byref(P(k=31)), None, ctypes.byref(t), None,
                                 None) == abi.HM_EINVAL  # Bloom needed
    b = abi.Bloom(None, 0, 4)
    assert L.hm_bloom_insert_occ(ctypes.byref(good), ctypes.byref(P(k=31, flags=abi.HM_BLOOM_IN_TABLE)),
                                 ctypes.byref(b), ctypes.byref(t), None, None) == abi.HM_EINVAL
    assert "list" in abi.last_error()
    # the card pass with a stream: a bad stream is rejected after the sketch's own checks
    tab = abi.Table(64, 1024, 0, 31, 64, None)
    c = abi.Card(64, 14, 10, 8, 0, 64, tab, tab)
    r = abi.Reads(8, 8, 8, None, 1, 100, 100)
    assert L.hm_cardinality_occ(ctypes.byref(r), ctypes.byref(P(k=31)), ctypes.byref(c), ctypes.byref(o),
                                None) == abi.HM_EINVAL
    assert "aligned" in abi.last_error()
    assert L.hm_cardinality_occ(ctypes.byref(r), ctypes.byref(P(k=31)), ctypes.byref(c), None,
                                None) == abi.HM_EINVAL


def test_binned_path_rejections(L):
    """The binned path's entry points check their arguments on the host: scratch sizes follow the
    formula in the header, and bad bins, reads, k or flags return HM_EINVAL before any launch."""
    assert L.hm_bins_scratch_bytes(0, 0) == (1 << 27) + 8 * (2050 + 2) + 4096 + 32
    assert L.hm_bins_scratch_bytes(9, 10) == (1 << 27) + 8 * (2050 + 2 * 512) + 4096 * 512 + 32 * (1 << 19)
    assert L.hm_bins_scratch_bytes(11, 0) == 0 and L.hm_bins_scratch_bytes(0, 12) == 0
    assert L.hm_bins_scratch_bytes(0, 11) > 0
    # capacity: the windows plus the padding of every range of either level (7 records a range in the
    # first, 3 in the second), whichever is more
    assert L.hm_bins_capacity(1000, 2, 3) == 1000 + max(7 * 1024 * 4, 3 * 8 * 32)
    assert L.hm_bins_capacity(10 ** 9, 9, 11) == 10 ** 9 + 3 * 8 * (1 << 20)
    assert L.hm_bins_capacity(5, 11, 0) == 0 and L.hm_bins_capacity(5, 0, 12) == 0
    good = dict(recs=256, tmp=512, capacity=1000 + 7 * 4096, group_bits=2, bin_bits=3, scratch=1024, bin_start=2048,
                status=4096, stats=None)
    r = abi.Reads(8, 8, 8, None, 10, 1000, 100)
    for bad, msg in ((dict(recs=None), "NULL"), (dict(status=None), "NULL"), (dict(recs=264), "aligned"), (dict(scratch=1032), "aligned"),
                     (dict(group_bits=11), "at most"), (dict(bin_bits=12), "at most"),
                     (dict(capacity=1000), "padding"), (dict(tmp=576), "aligned")):
        b = abi.Bins(**dict(good, **bad))
        assert L.hm_bin_kmers(ctypes.byref(r), ctypes.byref(P(k=21)), ctypes.byref(b), 0, None) == abi.HM_EINVAL
        assert msg in abi.last_error(), (bad, abi.last_error())
    b = abi.Bins(**good)
    assert L.hm_bin_kmers(ctypes.byref(r), ctypes.byref(P(k=63)), ctypes.byref(b), 0, None) == abi.HM_EINVAL
    assert "k <= 61" in abi.last_error()
    rv = abi.Reads(8, 8, 8, 8, 10, 1000, 0)  # read offsets: variable-length reads
    assert L.hm_bin_kmers(ctypes.byref(rv), ctypes.byref(P(k=21)), ctypes.byref(b), 0, None) == abi.HM_EINVAL
    assert "fixed-length" in abi.last_error()
    big = abi.Bins(**dict(good, capacity=1 << 40))
    rb = abi.Reads(8, 8, 8, None, 1 << 26, 150 << 26, 150)  # 2^26 reads x 130 windows >= 2^32
    assert L.hm_bin_kmers(ctypes.byref(rb), ctypes.byref(P(k=21)), ctypes.byref(big), 0, None) == abi.HM_EINVAL
    assert "2^32" in abi.last_error()
    assert L.hm_bin_kmers(ctypes.byref(r), ctypes.byref(P(k=21)), ctypes.byref(b), 2, None) == abi.HM_EINVAL
    assert "flags" in abi.last_error()
    # the card pass that counts the first level's histogram: the sketch's checks, then the bins'
    tab = abi.Table(64, 1024, 0, 21, 64, None)
    c = abi.Card(64, 14, 10, 8, 0, 64, tab, tab)
    cb = abi.Bins(**dict(good, recs=None))
    assert L.hm_cardinality_bins(ctypes.byref(r), ctypes.byref(P(k=21)), ctypes.byref(c), ctypes.byref(cb),
                                 None) == abi.HM_EINVAL
    assert "NULL" in abi.last_error()
    assert L.hm_cardinality_bins(ctypes.byref(rv), ctypes.byref(P(k=21)), ctypes.byref(c), ctypes.byref(b),
                                 None) == abi.HM_EINVAL
    assert "fixed-length" in abi.last_error()
    c16 = abi.Card(64, 16, 10, 8, 0, 64, tab, tab)  # 64 KiB of registers leave no room for the groups
    assert L.hm_cardinality_bins(ctypes.byref(r), ctypes.byref(P(k=21)), ctypes.byref(c16), ctypes.byref(b),
                                 None) == abi.HM_EINVAL
    assert "64 KiB" in abi.last_error()
    # HM_BINS_COUNTED is taken only after a matching hm_cardinality_bins (noted on the host); with no
    # reads hm_cardinality_bins launches nothing (its acceptance is a GPU test: it clears device words)
    r0 = abi.Reads(8, 8, 8, None, 0, 0, 100)
    assert L.hm_bin_kmers(ctypes.byref(r0), ctypes.byref(P(k=21)), ctypes.byref(b), abi.HM_BINS_COUNTED,
                          None) == abi.HM_EINVAL
    assert "HM_BINS_COUNTED" in abi.last_error()
    assert L.hm_cardinality_bins(ctypes.byref(r0), ctypes.byref(P(k=21)), ctypes.byref(c), ctypes.byref(b), None) == 0
    other = abi.Bins(**dict(good, bin_bits=4))
    assert L.hm_bin_kmers(ctypes.byref(r0), ctypes.byref(P(k=21)), ctypes.byref(other), abi.HM_BINS_COUNTED,
                          None) == abi.HM_EINVAL  # same scratch, other bin count: the note is taken and refused
    assert L.hm_bin_kmers(ctypes.byref(r0), ctypes.byref(P(k=21)), ctypes.byref(b), abi.HM_BINS_COUNTED,
                          None) == abi.HM_EINVAL  # ... and gone
    # partition of a stream: the stream's checks, k, and room for the stream's capacity, before any launch
    so = abi.Occ(64, 64, 1000, 64)
    assert L.hm_bin_occ(ctypes.byref(abi.Occ(64, 64, 10, None)), ctypes.byref(P(k=21)), ctypes.byref(b),
                        None) == abi.HM_EINVAL
    assert L.hm_bin_occ(ctypes.byref(so), ctypes.byref(P(k=63)), ctypes.byref(b), None) == abi.HM_EINVAL
    assert "k <= 61" in abi.last_error()
    assert L.hm_bin_occ(ctypes.byref(abi.Occ(64, 64, 5000, 64)), ctypes.byref(P(k=21)), ctypes.byref(b),
                        None) == abi.HM_EINVAL  # 5000 entries and their padding do not fit 1000 + 7 * 4096
    assert "stream" in abi.last_error()
    assert L.hm_bin_occ(ctypes.byref(abi.Occ(64, 64, 1 << 32, 64)), ctypes.byref(P(k=21)), ctypes.byref(big),
                        None) == abi.HM_EINVAL
    assert "2^32" in abi.last_error()
    e = abi.Export(64, 64, 64, 64, 64, 64, 64, 10, 64, None, 2, 2, None, 0)
    o = abi.Occ(64, 64, 10, 64)
    assert L.hm_count_bins(ctypes.byref(b), ctypes.byref(P(k=21)), abi.HM_EXPORT_SORTED, ctypes.byref(e),
                           ctypes.byref(o), None) == abi.HM_EINVAL
    assert L.hm_count_bins(ctypes.byref(b), ctypes.byref(P(k=21)), 0, ctypes.byref(e), None, None) == abi.HM_EINVAL
    assert L.hm_count_bins(ctypes.byref(b), ctypes.byref(P(k=63)), 0, ctypes.byref(e), ctypes.byref(o),
                           None) == abi.HM_EINVAL
    assert L.hm_export_merge(None, ctypes.byref(e), 64, None) == abi.HM_EINVAL
    assert L.hm_export_merge(ctypes.byref(e), ctypes.byref(e), None, None) == abi.HM_EINVAL


def test_bin_plan_keeps_bins_within_their_local_limits():
    """plan_bins: enough bins that a bin's expected distinct k-mers and inserted k-mers stay well
    inside the deferred list (2048) and the table's spill limit (384), up to 2^21 bins, with the
    second level taking at least half of the bits (at most 11); 2^20 bins while a bin stays within
    25% of the targets."""
    from paper_1705_11147_amd.kmer import plan_bins
    for distinct, seen2, bypass in ((4.76e8, 1.03e8, False), (4.4e6, 1.1e6, False), (1e3, 500, False),
                                    (4.76e8, 1.03e8, True), (1.2e9, 2.5e8, False), (10, 2, False), (3e9, 9e8, True)):
        g, b = plan_bins(distinct, seen2, bypass)
        assert 0 <= g <= 10 and 0 <= b <= 11 and (b >= g or b == 11)
        bins = 1 << (g + b)
        inserted = (distinct if bypass else seen2) / bins
        assert distinct / bins <= 900 and inserted <= 192 or g + b == 21 or \
            (g + b == 20 and distinct / bins <= 1.25 * 900 and inserted <= 1.25 * 192)
        if g + b > 0:  # not more bins than needed: half as many would break a limit
            half = bins / 2
            assert distinct / half > 900 or (distinct if bypass else seen2) / half > 192
    assert plan_bins(4.76e8, 1.03e8) == (9, 11)
    assert plan_bins(1.096e9, 2.1e8) == (9, 11)  # the human-scale share: 16% past the targets at 2^20
    assert plan_bins(1.2e9, 2.5e8) == (10, 11)  # 27% past them: 2^21


def test_status_code_maps_words_on_the_host(L):
    """hm_status_code maps a status word already on the host to the code hm_status returns:
    errors by severity (timeout, overflow, capacity, output), the classification bit alone is
    no error."""
    assert L.hm_status_code(0) == abi.HM_OK
    assert L.hm_status_code(abi.HM_ST_CLASSIFIED) == abi.HM_OK
    assert L.hm_status_code(abi.HM_ST_TABLE_FULL) == abi.HM_ECAPACITY
    assert "count table" in abi.last_error()
    assert L.hm_status_code(abi.HM_ST_LIST_FULL | abi.HM_ST_CLASSIFIED) == abi.HM_ECAPACITY
    assert "first-occurrence list" in abi.last_error()
    assert L.hm_status_code(abi.HM_ST_STREAM_FULL) == abi.HM_ECAPACITY
    assert "occurrence stream" in abi.last_error()
    assert L.hm_status_code(abi.HM_ST_OUTPUT_FULL) == abi.HM_EOUTPUT
    assert L.hm_status_code(abi.HM_ST_OUTPUT_FULL | abi.HM_ST_TABLE_FULL) == abi.HM_ECAPACITY
    assert L.hm_status_code(abi.HM_ST_OVERFLOW | abi.HM_ST_TABLE_FULL) == abi.HM_EOVERFLOW
    assert L.hm_status_code(abi.HM_ST_TIMEOUT | abi.HM_ST_OVERFLOW) == abi.HM_ETIMEOUT


def test_random_access_rejects(L):
    assert L.hm_random_access(None, 1024, 0, 10, 1, 8, None) == abi.HM_EINVAL
    assert L.hm_random_access(8, 1000, 0, 10, 1, 8, None) == abi.HM_EINVAL
    assert L.hm_random_access(8, 1024, 9, 10, 1, 8, None) == abi.HM_EINVAL
    assert L.hm_random_access(8, 1024, abi.HM_RA_COPY | abi.HM_RA_SERIAL, 10, 1, 8, None) == abi.HM_EINVAL


def test_package_import_is_lazy_and_loud():
    import subprocess
    import sys
    code = ("import paper_1705_11147_amd.abi as a; a._build.SO='/nonexistent/lib.so'; a._LIB=None\n"
            "try:\n a.lib()\nexcept RuntimeError as e:\n print('loud', e)\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert "loud" in out.stdout


# ---- the ctypes mirror against the C header, compiled by gcc

C_NAMES = {"Reads": "hm_reads_t", "Params": "hm_params_t", "Table": "hm_table_t", "Bloom": "hm_bloom_t",
           "List": "hm_list_t", "Export": "hm_export_t", "Card": "hm_card_t", "CardSummary": "hm_card_summary_t",
           "Contigs": "hm_contigs_t", "Occ": "hm_occ_t", "Bins": "hm_bins_t", "BatchSet": "hm_batch_set_t",
           "BatchTuning": "hm_batch_tuning_t", "BatchPlan": "hm_batch_plan_t"}


def test_struct_layout_matches_header(tmp_path):
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hm_kmer.h"', "int main(void) {"]
    expect = []
    for py, c in C_NAMES.items():
        cls = getattr(abi, py)
        lines.append('printf("%%zu\\n", sizeof(%s));' % c)
        expect.append(("sizeof " + c, ctypes.sizeof(cls)))
        for name, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (c, name))
            expect.append(("%s.%s" % (c, name), getattr(cls, name).offset))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE, "-I",
                    os.path.join(rocm, "include"), str(src), "-o", str(exe)], check=True, capture_output=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert len(got) == len(expect)
    bad = [(what, c, py) for (what, py), c in zip(expect, got) if c != py]
    assert not bad, "C vs ctypes: %r" % bad


def test_sorted_export_scratch_and_rejections(L):
    # scratch: keys, indices and staged counters (88 B per record), tile counts, digit totals
    assert L.hm_export_sort_bytes(1 << 20) == (88 << 20) + 1024 * 256 + 1024 + 4 * 65537 + 252
    assert L.hm_export_sort_bytes(10) >= 88 * 10 + 2048
    t = abi.Table(64, 1024, 0, 31, 64, None)
    S = abi.HM_EXPORT_SORTED

    def ex(cap=10, work=None, nbytes=0):
        return abi.Export(8, 8, 8, 16, 16, 8, 8, cap, 64, None, 0, 0, work, nbytes)
    assert L.hm_export_table(ctypes.byref(t), S, ctypes.byref(ex()), None) == abi.HM_EINVAL  # no scratch
    need = L.hm_export_sort_bytes(10)
    assert L.hm_export_table(ctypes.byref(t), S, ctypes.byref(ex(work=4096 + 64, nbytes=need)),
                             None) == abi.HM_EINVAL  # misaligned
    assert L.hm_export_table(ctypes.byref(t), S, ctypes.byref(ex(work=4096, nbytes=need - 1)),
                             None) == abi.HM_EINVAL  # too small
    assert L.hm_export_table(ctypes.byref(t), S, ctypes.byref(ex(cap=1 << 32, work=4096, nbytes=1 << 62)),
                             None) == abi.HM_EINVAL  # indices are 32-bit
    assert "SORTED" in abi.last_error()


def test_heavy_list_rejections(L):
    t = abi.Table(64, 1024, 0, 31, 64, None, None, abi.HM_MAX_HEAVY + 1, 0)
    r = abi.Reads(8, 8, 8, None, 1, 100, 100)
    p = P(k=31, flags=abi.HM_BLOOM_BYPASS)
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(p), None, ctypes.byref(t), None, None) == abi.HM_EINVAL
    t = abi.Table(64, 1024, 0, 31, 64, None, None, 3, 0)  # keys NULL
    assert L.hm_bloom_insert(ctypes.byref(r), ctypes.byref(p), None, ctypes.byref(t), None, None) == abi.HM_EINVAL
    assert "heavy" in abi.last_error()


def test_contigs_scratch_and_rejections(L):
    """hm_contigs_work_bytes and the host-side checks of hm_contigs (no device call)."""
    assert L.hm_contigs_work_bytes(0) > 0
    w = L.hm_contigs_work_bytes(1 << 20)
    assert w == 186 * (1 << 20) + 512  # 186 bytes per record and the control block
    assert L.hm_contigs_work_bytes(1 << 29) == 0  # too many records
    e = abi.Export(8, 8, None, None, None, 8, 8, 1000, 8, None)
    c = abi.Contigs(8, 100, 8, 10, 8, 8, 256, w)
    assert L.hm_contigs(ctypes.byref(e), 20, 0, ctypes.byref(c), None) == abi.HM_EINVAL  # even k, canonical
    assert L.hm_contigs(ctypes.byref(e), 0, abi.HM_FORWARD_ONLY, ctypes.byref(c), None) == abi.HM_EINVAL
    assert L.hm_contigs(ctypes.byref(e), 21, 4, ctypes.byref(c), None) == abi.HM_EINVAL  # unknown flag
    assert L.hm_contigs(None, 21, 0, ctypes.byref(c), None) == abi.HM_EINVAL
    e2 = abi.Export(8, 8, None, None, None, 8, 8, 1 << 29, 8, None)
    assert L.hm_contigs(ctypes.byref(e2), 21, 0, ctypes.byref(c), None) == abi.HM_EINVAL  # too many records
    e3 = abi.Export(None, 8, None, None, None, 8, 8, 1000, 8, None)
    assert L.hm_contigs(ctypes.byref(e3), 21, 0, ctypes.byref(c), None) == abi.HM_EINVAL  # no keys
    c2 = abi.Contigs(8, 100, 8, 10, 8, 8, 264, w)
    assert L.hm_contigs(ctypes.byref(e), 21, 0, ctypes.byref(c2), None) == abi.HM_EINVAL  # misaligned work
    c3 = abi.Contigs(8, 100, 8, 10, 8, 8, 256, L.hm_contigs_work_bytes(1000) - 1)
    assert L.hm_contigs(ctypes.byref(e), 21, 0, ctypes.byref(c3), None) == abi.HM_EINVAL  # work too small
    c4 = abi.Contigs(None, 100, 8, 10, 8, 8, 256, w)
    assert L.hm_contigs(ctypes.byref(e), 21, 0, ctypes.byref(c4), None) == abi.HM_EINVAL  # no seq
    assert abi.last_error()


@pytest.mark.parametrize("bad", [dict(blocks_per_cu=0), dict(blocks_per_cu=17), dict(tile_bases=1023),
                                 dict(tile_bases=262145), dict(list_per_item=255), dict(slots_per_item=3000),
                                 dict(set_major=65)])
def test_batch_tuning_rejections(L, bad):
    """hm_batch_prepare checks the tuning on the host before any device call."""
    tu = dict(blocks_per_cu=8, tile_bases=65536, list_per_item=65536, slots_per_item=65536, set_major=2)
    tu.update(bad)
    sets = (abi.BatchSet * 1)()
    plan = abi.BatchPlan()
    work = 1 << 20  # never dereferenced: the call fails first
    rc = L.hm_batch_prepare(sets, 1, ctypes.byref(P()), 0, 20, 0, ctypes.byref(abi.BatchTuning(**tu)), work,
                            L.hm_batch_work_bytes(1), ctypes.byref(plan), None)
    assert rc == abi.HM_EINVAL and abi.last_error()


@pytest.mark.parametrize("read_len,tile_bases", [(2000, 1024), (16321, 262144)])
def test_batch_read_length_rejections(L, read_len, tile_bases):
    """A read longer than a pass-1 item, or than one LDS run of an item, is refused on the host."""
    sets = (abi.BatchSet * 1)()
    sets[0].n_reads, sets[0].read_len = 10, read_len
    tu = abi.BatchTuning(8, tile_bases, 65536, 65536, 2)
    plan = abi.BatchPlan()
    rc = L.hm_batch_prepare(sets, 1, ctypes.byref(P()), 0, 20, 0, ctypes.byref(tu), 1 << 20,
                            L.hm_batch_work_bytes(1), ctypes.byref(plan), None)
    assert rc == abi.HM_EINVAL and "read_len" in abi.last_error()
