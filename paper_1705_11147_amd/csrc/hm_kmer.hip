// HIP kernels and C ABI of the k-mer analysis path for MI355X (gfx950).
//
// Method: arXiv 1705.11147, section "The Meraculous Assembly Pipeline"
// (step 1, k-mer analysis) and section "Parallel k-mer analysis" (Bloom
// filter in front of the count table, extension counters, thresholds).
// The argument conventions are documented in include/hm_kmer.h.
//
// Design (one GPU, HBM-resident data):
//   * hm_pack_reads turns ASCII bases + Phred bytes into 2-bit codes and two
//     bit masks (invalid base, high-quality base): 0.5 byte per base, read
//     twice less than the ASCII input.
//   * Pass 1 stages tiles of packed reads in LDS and extracts every window
//     with funnel shifts (forward code) and a 2-bit group reversal (reverse
//     complement).  Each occurrence first probes the open-addressing table
//     with loads; if its k-mer is there it is counted at once.  Otherwise it
//     does one device-scope atomic OR on one 64-bit Bloom word: a k-mer the
//     filter has seen is inserted and counted, an unseen one (exactly one
//     occurrence per distinct k-mer, unless a false positive) goes to a
//     first-occurrence list.  Random atomics are the scarce resource on this
//     path (a few 10^10 per second), so hits skip the Bloom atomic.
//   * Pass 2 walks that list and counts the entries whose k-mer made it into
//     the table.  Every occurrence is therefore counted exactly once, so the
//     final table equals the plain definition whatever the false positives.
//   * Slots are 64 bytes (two per 128-byte cache line): two key words, each
//     carrying a "written" bit so a reader can tell a half-published two-word
//     key from a complete one without fences; a word of nine 7-bit narrow
//     counters (no left extension, left A..T, right A..T); u32 wide counters
//     nl, tl[4], tr[4]; and a 32-bit word that is the Bloom filter word of the
//     keys homed at the slot until classification.  A hit costs one 64-bit CAS
//     on the narrow word, which the probe's 16-byte load returned together
//     with the first key word; a lane about to pass 127, or a CAS that keeps
//     losing to others (a hot key), moves the slot to the wide counters (two
//     atomic adds per later occurrence).  count = nl + sum(tl), narrow + wide.
//   * With an owner filter (one share of a sharded run) the cardinality pass
//     can write the owned occurrences to a stream, and pass 1 then reads that
//     stream (k_pass1_stream) instead of scanning every window again.
#include "hm_device.h"

namespace hm {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) { return fail(HM_EHIP, "%s: %s", what, hipGetErrorString(e)); }

static std::atomic<int> g_cus[64];

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = g_cus[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        g_cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

uint64_t grid_for(uint64_t items, int per_cu) {
    const uint64_t blocks = (items + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)device_cus() * per_cu;
    return blocks < 1 ? 1 : (blocks < cap ? blocks : cap);
}

}  // namespace hm

namespace {

using namespace hm;

// Pass 1 over fixed-length reads: tiles of whole reads staged in LDS.  HEAVY:
// the table's heavy keys are counted in dynamic LDS and flushed at the end.
template <int KW, bool CHECKED, bool HEAVY>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_pass1_fixed(PassArgs a, int32_t reads_per_tile, int64_t n_tiles) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    extern __shared__ uint64_t s_heavy[];
    HeavyLds hv{};
    if (HEAVY) hv = heavy_setup(a, s_heavy);
    ListCursor cur{0, kListChunk};
    Stats st = {};
    const bool seen_all = classified_in_table(a);
    fixed_windows<true>(a, reads_per_tile, n_tiles, s_b2, s_nm, s_hq, [&](bool act, const Occ &o, int64_t) {
        pass1_occ<KW, CHECKED, kListChunk, HEAVY>(a, act, o, cur, st, &hv, seen_all);
    });
    list_close(a, cur);
    if (HEAVY) heavy_flush<KW, CHECKED>(a, hv);
    stats_flush(a.stats, st);
}

// Pass 1 over fixed-length reads with an owner filter: owned occurrences are
// queued in LDS and counted with every lane of the workgroup busy.
template <int KW, bool CHECKED, bool HEAVY>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_pass1_owned(PassArgs a, int32_t reads_per_tile,
                                                                       int64_t n_tiles) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    __shared__ uint4 s_qkey[kQueue];
    __shared__ uint8_t s_qext[kQueue];
    __shared__ unsigned s_qn;
    __shared__ int s_stop;
    extern __shared__ uint64_t s_heavy[];
    HeavyLds hv{};
    if (HEAVY) hv = heavy_setup(a, s_heavy);
    ListCursor cur{0, kListChunk};
    Stats st = {};
    const bool seen_all = classified_in_table(a);
    const OccQueue q{s_qkey, s_qext, &s_qn, &s_stop};
    fixed_windows_queued<true>(a, reads_per_tile, n_tiles, s_b2, s_nm, s_hq, q, [&](bool act, const Occ &o, int64_t) {
        pass1_occ<KW, CHECKED, kListChunk, HEAVY>(a, act, o, cur, st, &hv, seen_all);
    });
    list_close(a, cur);
    if (HEAVY) heavy_flush<KW, CHECKED>(a, hv);
    stats_flush(a.stats, st);
}

// Pass 1 over variable-length reads (read_off given).
template <int KW, bool CHECKED, bool HEAVY>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_pass1_var(PassArgs a, int64_t n_tiles) {
    __shared__ int64_t s_off[kVarReads + 1];
    __shared__ int64_t s_pre[kVarReads + 1];
    extern __shared__ uint64_t s_heavy[];
    HeavyLds hv{};
    if (HEAVY) hv = heavy_setup(a, s_heavy);
    ListCursor cur{0, kListChunk};
    Stats st = {};
    const bool seen_all = classified_in_table(a);
    var_windows<true>(a, n_tiles, s_off, s_pre, [&](bool act, const Occ &o, int64_t) {
        pass1_occ<KW, CHECKED, kListChunk, HEAVY>(a, act, o, cur, st, &hv, seen_all);
    });
    list_close(a, cur);
    if (HEAVY) heavy_flush<KW, CHECKED>(a, hv);
    stats_flush(a.stats, st);
}

// Pass 1 over an owned-occurrence stream (hm_bloom_insert_occ): one entry per
// lane, grid-stride with a wave-uniform trip count (pass1_occ appends to the
// first-occurrence list a wave at a time); holes are skipped.
template <int KW, bool CHECKED, bool HEAVY>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_pass1_stream(PassArgs a, const uint64_t *keys,
                                                                        const uint8_t *ext,
                                                                        const unsigned long long *count, uint64_t cap) {
    extern __shared__ uint64_t s_heavy[];
    const uint64_t n = *count;  // written by earlier kernels on the stream
    if (n > cap) {  // entries were dropped: the stream is void
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(a.status, HM_ST_STREAM_FULL);
        return;
    }
    HeavyLds hv{};
    if (HEAVY) hv = heavy_setup(a, s_heavy);
    ListCursor cur{0, kListChunk};
    Stats st = {};
    const bool seen_all = classified_in_table(a);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock; i0 < n; i0 += stride) {
        if (aborted(a.status)) break;  // wave-uniform
        const uint64_t i = i0 + threadIdx.x;
        Occ o{0, 0, 4, 4};
        bool act = false;
        if (i < n) {
            const uint8_t e = ext[i];
            if (e != kHole) {
                const uint4 kk = *reinterpret_cast<const uint4 *>(keys + 2 * i);
                o.hi = ((uint64_t)kk.y << 32) | kk.x;
                o.lo = ((uint64_t)kk.w << 32) | kk.z;
                o.left = e & 15;
                o.right = e >> 4;
                act = true;
            }
        }
        pass1_occ<KW, CHECKED, kListChunk, HEAVY>(a, act, o, cur, st, &hv, seen_all);
    }
    list_close(a, cur);
    if (HEAVY) heavy_flush<KW, CHECKED>(a, hv);
    stats_flush(a.stats, st);
}

// Pass 2: count the first occurrences whose k-mer is in the table.
template <int KW, bool CHECKED>
__global__ __launch_bounds__(kBlock) void k_pass2(PassArgs a) {
    if (*a.status & kAbortBits) return;  // pass 1 failed; the table is rebuilt by the caller
    const uint64_t n = min((uint64_t)*a.lcount, a.lcap);
    Stats st = {};
    // uniform trip count per wave so the counters can be summed with shuffles at the end
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock; i0 < n; i0 += stride) {
        const uint64_t i = i0 + threadIdx.x;
        if (i >= n) continue;
        const uint8_t e = a.lext[i];
        if (e == kHole) continue;
        pass2_entry<KW, CHECKED>(a, a.lkeys[2 * i], a.lkeys[2 * i + 1], e, st);
    }
    stats_flush(a.stats, st);
}

__global__ __launch_bounds__(kBlock) void k_classify(Slot *slots, uint64_t cap, uint32_t min_depth, uint32_t ext_min,
                                                     uint32_t *status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, HM_ST_CLASSIFIED);  // the filter words are gone
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * kBlock) {
        Slot *s = slots + i;
        if (s->a == 0) continue;
        uint32_t tl[4], tr[4];
        const uint64_t cnt = slot_counts(s, tl, tr);
        const uint32_t kept = cnt >= min_depth ? 1u : 0u;
        const uint32_t ovf = cnt > 0xFFFFFFFFull ? 1u : 0u;
        s->cls = side_class(tl, ext_min) | (side_class(tr, ext_min) << 8) | (kept << 16) | (ovf << 17);
    }
}

// PER slots per lane: a chunk of 64 * PER slots per wave and one output-counter
// atomic per chunk.  The plain export takes 2048-slot chunks (a quarter of the
// atomics on the one counter); the key-ordered one keeps 512, whose record runs
// its sort's grouping passes were measured faster on.
template <int KW, int PER>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_export(const Slot *slots, uint64_t cap, uint32_t flags, hm_export_t out,
                                                   uint32_t *status, uint4 *staged) {
    constexpr int kChunk = 64 * PER;
    __shared__ uint16_t s_rank[kBlock / 64][kChunk];
    uint64_t dsum = 0, dxor = 0;
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * kBlock) >> 6;
    for (uint64_t first = wave * kChunk; first < cap; first += n_waves * kChunk)
        export_chunk<KW, PER>(slots, first, cap, flags, out, status, s_rank[threadIdx.x >> 6], dsum, dxor, staged);
    digest_flush(out, dsum, dxor);
}

__global__ __launch_bounds__(kBlock) void k_pack(const uint8_t *ascii, const uint8_t *qual, int64_t n_bases,
                                                 uint64_t n_mask_words, int qual_offset, int qcut, uint64_t *b2,
                                                 uint64_t *nm, uint64_t *hq) {
    const bool aligned = ((((uintptr_t)ascii) | ((uintptr_t)qual)) & 15) == 0;
    for (uint64_t m = (uint64_t)blockIdx.x * kBlock + threadIdx.x; m < n_mask_words;
         m += (uint64_t)gridDim.x * kBlock) {
        const int64_t base = (int64_t)m * 64;
        uint64_t c0 = 0, c1 = 0, nmask = ~0ull, hmask = 0;
        if (base < n_bases) {
            const int cnt = (int)min((int64_t)64, n_bases - base);
            nmask = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nv = cnt - 16 * v;
                uint4 sa = make_uint4(0, 0, 0, 0), sq = make_uint4(0, 0, 0, 0);
                if (nv >= 16 && aligned) {
                    sa = *reinterpret_cast<const uint4 *>(ascii + base + 16 * v);
                    sq = *reinterpret_cast<const uint4 *>(qual + base + 16 * v);
                } else if (nv > 0) {
                    uint32_t ta[4] = {0, 0, 0, 0}, tq[4] = {0, 0, 0, 0};
                    for (int i = 0; i < 16 && i < nv; ++i) {
                        ta[i >> 2] |= (uint32_t)ascii[base + 16 * v + i] << (8 * (i & 3));
                        tq[i >> 2] |= (uint32_t)qual[base + 16 * v + i] << (8 * (i & 3));
                    }
                    sa = make_uint4(ta[0], ta[1], ta[2], ta[3]);
                    sq = make_uint4(tq[0], tq[1], tq[2], tq[3]);
                }
                uint64_t codes;
                uint32_t bad, good;
                pack16(sa, sq, nv, qual_offset, qcut, codes, bad, good);
                if (v < 2) c0 |= codes << (32 * (1 - v));
                else c1 |= codes << (32 * (3 - v));
                nmask |= (uint64_t)bad << (16 * (3 - v));
                hmask |= (uint64_t)good << (16 * (3 - v));
            }
        }
        b2[2 * m] = c0;
        b2[2 * m + 1] = c1;
        nm[m] = nmask;
        hq[m] = hmask;
    }
}

}  // namespace

namespace hm {

int check_reads(const hm_reads_t *r, int k) {
    if (!r) return fail(HM_EINVAL, "reads is NULL");
    if (r->n_reads < 0 || r->n_bases < 0) return fail(HM_EINVAL, "negative read or base count");
    if (r->n_reads == 0) return HM_OK;
    if (!r->bases2 || !r->nmask || !r->hqmask) return fail(HM_EINVAL, "packed read pointers are NULL");
    if (!r->read_off) {
        if (r->read_len <= 0) return fail(HM_EINVAL, "read_len must be > 0 when read_off is NULL");
        if (r->n_reads > r->n_bases / r->read_len) return fail(HM_EINVAL, "n_reads * read_len exceeds n_bases");
    }
    (void)k;
    return HM_OK;
}

int check_occ(const hm_occ_t *o) {
    if (!o || !o->count) return fail(HM_EINVAL, "occurrence stream or its counter is NULL");
    if (o->capacity > 0 && (!o->keys || !o->ext)) return fail(HM_EINVAL, "occurrence stream arrays are NULL");
    if (((uintptr_t)o->keys) & 15) return fail(HM_EINVAL, "occurrence stream keys must be 16-byte aligned");
    return HM_OK;
}

int check_table(const hm_table_t *t) {
    if (!t || !t->slots || !t->status) return fail(HM_EINVAL, "table or its buffers are NULL");
    if (!pow2(t->capacity)) return fail(HM_EINVAL, "table capacity must be a power of two");
    if (((uintptr_t)t->slots) & 63) return fail(HM_EINVAL, "table slots must be 64-byte aligned");
    return HM_OK;
}

}  // namespace hm

// ====================================================================== C ABI

extern "C" {

int hm_abi_version(void) { return HM_ABI_VERSION; }

const char *hm_last_error(void) { return hm::g_err; }

uint64_t hm_mask_words(int64_t n_bases) { return (uint64_t)(n_bases < 0 ? 0 : n_bases) / 64 + 3; }

uint64_t hm_bases2_words(int64_t n_bases) { return 2 * hm_mask_words(n_bases); }

size_t hm_table_bytes(uint64_t capacity) { return (size_t)capacity * HM_SLOT_BYTES; }

size_t hm_bloom_bytes(uint64_t n_words) { return (size_t)n_words * 8; }

size_t hm_list_bytes(uint64_t capacity) { return (size_t)capacity * 17; }

size_t hm_occ_bytes(uint64_t capacity) { return (size_t)capacity * 17; }

int hm_check_params(const hm_params_t *p) {
    if (!p) return fail(HM_EINVAL, "params is NULL");
    if (p->k < 1 || p->k > 63) return fail(HM_EINVAL, "k must be in 1..63 (got %d)", p->k);
    if (!(p->flags & HM_FORWARD_ONLY) && (p->k % 2) == 0)
        return fail(HM_EINVAL, "k must be odd for canonical k-mers (got %d)", p->k);
    if (p->min_depth < 1) return fail(HM_EINVAL, "min_depth must be >= 1");
    if (p->ext_min < 1) return fail(HM_EINVAL, "ext_min must be >= 1");
    if (p->n_owners < 1 || p->owner >= p->n_owners) return fail(HM_EINVAL, "owner must be < n_owners");
    if (p->flags & ~(HM_FORWARD_ONLY | HM_BLOOM_BYPASS | HM_CHECKED | HM_BLOOM_IN_TABLE))
        return fail(HM_EINVAL, "unknown flags");
    return HM_OK;
}

int hm_table_init(hm_table_t *t, hipStream_t s) {
    int rc = check_table(t);
    if (rc) return rc;
    rc = fill<uint4>(reinterpret_cast<uint4 *>(t->slots), t->capacity * (HM_SLOT_BYTES / 16), make_uint4(0, 0, 0, 0), s);
    if (rc) return rc;
    if (t->stats) {
        rc = fill<uint64_t>(t->stats, HM_N_STATS, 0ull, s);
        if (rc) return rc;
    }
    return fill<uint32_t>(t->status, 1, 0u, s);
}

int hm_bloom_init(hm_bloom_t *b, hipStream_t s) {
    if (!b || !b->words || !pow2(b->n_words)) return fail(HM_EINVAL, "bloom: NULL words or n_words not a power of two");
    if (b->n_hash < 1 || b->n_hash > 8) return fail(HM_EINVAL, "bloom: n_hash must be 1..8");
    return fill<uint64_t>(b->words, b->n_words, 0ull, s);
}

int hm_list_init(hm_list_t *l, hipStream_t s) {
    if (!l || !l->count) return fail(HM_EINVAL, "list or its counter is NULL");
    if (l->present) {
        if (!pow2(l->present_words)) return fail(HM_EINVAL, "presence filter words must be a power of two");
        int rc = fill<uint64_t>(l->present, l->present_words, 0ull, s);
        if (rc) return rc;
    }
    return fill<uint64_t>(l->count, 1, 0ull, s);
}

int hm_occ_init(hm_occ_t *o, hipStream_t s) {
    int rc = check_occ(o);
    if (rc) return rc;
    return fill<uint64_t>(o->count, 1, 0ull, s);
}

int hm_status_code(uint32_t st) {
    if (st & HM_ST_TIMEOUT) return fail(HM_ETIMEOUT, "a batched-phase wait passed its bound (status 0x%x)", st);
    if (st & HM_ST_OVERFLOW) return fail(HM_EOVERFLOW, "a k-mer counter passed 2^32 - 1 (status 0x%x)", st);
    if (st & HM_ST_STREAM_FULL)
        return fail(HM_ECAPACITY, "occurrence stream overflowed before pass 1 (status 0x%x)", st);
    if (st & (HM_ST_TABLE_FULL | HM_ST_LIST_FULL))
        return fail(HM_ECAPACITY, "%s full (status 0x%x)", (st & HM_ST_TABLE_FULL) ? "count table" : "first-occurrence list",
                    st);
    if (st & HM_ST_OUTPUT_FULL) return fail(HM_EOUTPUT, "export buffer too small (status 0x%x)", st);
    return HM_OK;
}

int hm_status(const hm_table_t *t, hipStream_t s) {
    if (!t || !t->status) return fail(HM_EINVAL, "table status is NULL");
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t st = 0;
    e = hipMemcpy(&st, t->status, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status)");
    return hm_status_code(st);
}

int hm_pack_reads(const uint8_t *ascii, const uint8_t *qual, int64_t n_bases, uint8_t qual_offset, uint8_t qcut,
                  uint64_t *bases2, uint64_t *nmask, uint64_t *hqmask, hipStream_t s) {
    if (n_bases < 0) return fail(HM_EINVAL, "n_bases < 0");
    if (!bases2 || !nmask || !hqmask) return fail(HM_EINVAL, "output pointers are NULL");
    if (n_bases > 0 && (!ascii || !qual)) return fail(HM_EINVAL, "input pointers are NULL");
    const uint64_t nmw = hm_mask_words(n_bases);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)grid_for(nmw, 16)), dim3(kBlock), 0, s, ascii, qual, n_bases, nmw,
                       (int)qual_offset, (int)qcut, bases2, nmask, hqmask);
    HM_LAUNCH_CHECK("hm_pack_reads");
    return HM_OK;
}

static int make_args(const hm_reads_t *r, const hm_params_t *p, hm_bloom_t *b, hm_table_t *t, hm_list_t *l,
                     PassArgs &a, bool need_reads) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_table(t);
    if (rc) return rc;
    if (t->k != p->k) return fail(HM_EINVAL, "table built for k=%d, params have k=%d", t->k, p->k);
    if (need_reads) {
        rc = check_reads(r, p->k);
        if (rc) return rc;
    }
    memset(&a, 0, sizeof a);
    const bool bypass = (p->flags & HM_BLOOM_BYPASS) || p->min_depth == 1;
    if (r && need_reads) {
        a.b2 = r->bases2;
        a.nm = r->nmask;
        a.hq = r->hqmask;
        a.read_off = r->read_off;
        a.n_reads = r->n_reads;
        a.n_bases = r->n_bases;
        a.read_len = r->read_len;
    }
    a.k = p->k;
    a.forward_only = (p->flags & HM_FORWARD_ONLY) ? 1 : 0;
    a.n_owners = p->n_owners;
    a.owner = p->owner;
    a.seed = p->seed;
    a.bypass = bypass ? 1 : 0;
    if (!bypass && need_reads) {
        if (p->flags & HM_BLOOM_IN_TABLE) {
            if (!b || b->n_hash < 1 || b->n_hash > 8)
                return fail(HM_EINVAL, "a Bloom filter in the table needs 1..8 hashes (hm_bloom_t.n_hash)");
            a.bloom = nullptr;
            a.bloom_mask = 0;
        } else {
            if (!b || !b->words || !pow2(b->n_words) || b->n_hash < 1 || b->n_hash > 8)
                return fail(HM_EINVAL, "a Bloom filter (power-of-two words, 1..8 hashes) is needed unless bypassed");
            if (b->n_words > (1ull << 40)) return fail(HM_EINVAL, "bloom too large");
            a.bloom = b->words;
            a.bloom_mask = b->n_words - 1;
        }
        a.n_hash = b->n_hash;
    }
    if (!bypass || !need_reads) {
        if (!l || !l->keys || !l->ext || !l->count) return fail(HM_EINVAL, "first-occurrence list is NULL");
        a.lkeys = l->keys;
        a.lext = l->ext;
        a.lcap = l->capacity;
        a.lcount = reinterpret_cast<unsigned long long *>(l->count);
        if (l->present) {
            if (!pow2(l->present_words) || l->present_hash < 1 || l->present_hash > 8)
                return fail(HM_EINVAL, "presence filter: power-of-two words and 1..8 bits per key");
            a.present = l->present;
            a.present_mask = l->present_words - 1;
            a.present_hash = l->present_hash;
        }
    }
    a.slots = reinterpret_cast<Slot *>(t->slots);
    a.cmask = t->capacity - 1;
    const uint64_t mp = t->max_probe ? (uint64_t)t->max_probe : (uint64_t)kDefaultMaxProbe;
    a.max_probe = (uint32_t)(mp < t->capacity ? mp : t->capacity);
    a.status = t->status;
    a.stats = reinterpret_cast<unsigned long long *>(t->stats);
    if (t->n_heavy > HM_MAX_HEAVY) return fail(HM_EINVAL, "table: n_heavy must be <= %d", HM_MAX_HEAVY);
    if (t->n_heavy && !t->heavy) return fail(HM_EINVAL, "table: heavy keys are NULL");
    a.heavy = t->heavy;
    a.n_heavy = t->n_heavy;
    return HM_OK;
}

int hm_bloom_insert(const hm_reads_t *r, const hm_params_t *p, hm_bloom_t *b, hm_table_t *t, hm_list_t *l,
                    hipStream_t s) {
    PassArgs a;
    int rc = make_args(r, p, b, t, l, a, true);
    if (rc) return rc;
    if (r->n_reads == 0) return HM_OK;
    const bool two = p->k >= 32;
    const bool checked = (p->flags & HM_CHECKED) != 0;
    const bool heavy = a.n_heavy > 0;
    const size_t lds = heavy_lds_bytes(a.n_heavy);
    const int grid_cap = device_cus() * 8;
    if (!r->read_off && r->read_len <= kTileBases - 64) {
        if (r->read_len < p->k) return HM_OK;  // no windows
        const bool owned = p->n_owners > 1;     // most windows dropped: queue the owned ones
        const int32_t rpt = kTileBases / r->read_len;
        const int64_t n_tiles = (r->n_reads + rpt - 1) / rpt;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
#define LAUNCH_FIXED(KW, CH, HV)                                                                        \
    do {                                                                                                \
        if (owned) hipLaunchKernelGGL((k_pass1_owned<KW, CH, HV>), g, dim3(kBlock), lds, s, a, rpt, n_tiles); \
        else hipLaunchKernelGGL((k_pass1_fixed<KW, CH, HV>), g, dim3(kBlock), lds, s, a, rpt, n_tiles);  \
    } while (0)
#define LAUNCH_FIXED2(KW, CH) \
    do { if (heavy) LAUNCH_FIXED(KW, CH, true); else LAUNCH_FIXED(KW, CH, false); } while (0)
        if (two) { if (checked) LAUNCH_FIXED2(2, true); else LAUNCH_FIXED2(2, false); }
        else { if (checked) LAUNCH_FIXED2(1, true); else LAUNCH_FIXED2(1, false); }
#undef LAUNCH_FIXED2
#undef LAUNCH_FIXED
    } else {
        if (!r->read_off) return fail(HM_EINVAL, "reads longer than %d bases need read_off", kTileBases - 64);
        const int64_t n_tiles = (r->n_reads + kVarReads - 1) / kVarReads;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
#define LAUNCH_VAR(KW, CH, HV) hipLaunchKernelGGL((k_pass1_var<KW, CH, HV>), g, dim3(kBlock), lds, s, a, n_tiles)
#define LAUNCH_VAR2(KW, CH) do { if (heavy) LAUNCH_VAR(KW, CH, true); else LAUNCH_VAR(KW, CH, false); } while (0)
        if (two) { if (checked) LAUNCH_VAR2(2, true); else LAUNCH_VAR2(2, false); }
        else { if (checked) LAUNCH_VAR2(1, true); else LAUNCH_VAR2(1, false); }
#undef LAUNCH_VAR2
#undef LAUNCH_VAR
    }
    HM_LAUNCH_CHECK("hm_bloom_insert");
    return HM_OK;
}

int hm_bloom_insert_occ(const hm_occ_t *o, const hm_params_t *p, hm_bloom_t *b, hm_table_t *t, hm_list_t *l,
                        hipStream_t s) {
    int rc = check_occ(o);
    if (rc) return rc;
    // the Bloom filter and list are set up as for pass 1 over reads; the reads are the stream
    const hm_reads_t none = {nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
    PassArgs a;
    rc = make_args(&none, p, b, t, l, a, true);
    if (rc) return rc;
    const bool two = p->k >= 32;
    const bool checked = (p->flags & HM_CHECKED) != 0;
    const bool heavy = a.n_heavy > 0;
    const size_t lds = heavy_lds_bytes(a.n_heavy);
    const dim3 g((unsigned)(device_cus() * 8));
    const unsigned long long *cnt = reinterpret_cast<const unsigned long long *>(o->count);
#define LAUNCH_S(KW, CH, HV) \
    hipLaunchKernelGGL((k_pass1_stream<KW, CH, HV>), g, dim3(kBlock), lds, s, a, o->keys, o->ext, cnt, o->capacity)
#define LAUNCH_S2(KW, CH) do { if (heavy) LAUNCH_S(KW, CH, true); else LAUNCH_S(KW, CH, false); } while (0)
    if (two) { if (checked) LAUNCH_S2(2, true); else LAUNCH_S2(2, false); }
    else { if (checked) LAUNCH_S2(1, true); else LAUNCH_S2(1, false); }
#undef LAUNCH_S2
#undef LAUNCH_S
    HM_LAUNCH_CHECK("hm_bloom_insert_occ");
    return HM_OK;
}

int hm_kmer_count(const hm_reads_t *r, const hm_params_t *p, hm_table_t *t, hm_list_t *l, hipStream_t s) {
    (void)r;
    int rc = hm_check_params(p);
    if (rc) return rc;
    if ((p->flags & HM_BLOOM_BYPASS) || p->min_depth == 1) return HM_OK;  // pass 1 counted everything
    PassArgs a;
    rc = make_args(nullptr, p, nullptr, t, l, a, false);
    if (rc) return rc;
    const bool two = p->k >= 32;
    const bool checked = (p->flags & HM_CHECKED) != 0;
    const dim3 g((unsigned)grid_for(l->capacity, 8));
#define LAUNCH2(KW, CH) hipLaunchKernelGGL((k_pass2<KW, CH>), g, dim3(kBlock), 0, s, a)
    if (two) { if (checked) LAUNCH2(2, true); else LAUNCH2(2, false); }
    else { if (checked) LAUNCH2(1, true); else LAUNCH2(1, false); }
#undef LAUNCH2
    HM_LAUNCH_CHECK("hm_kmer_count");
    return HM_OK;
}

int hm_classify_ext(const hm_params_t *p, hm_table_t *t, hipStream_t s) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_table(t);
    if (rc) return rc;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)grid_for(t->capacity, 16)), dim3(kBlock), 0, s,
                       reinterpret_cast<Slot *>(t->slots), t->capacity, p->min_depth, p->ext_min, t->status);
    HM_LAUNCH_CHECK("hm_classify_ext");
    return HM_OK;
}

int hm_export_table(const hm_table_t *t, uint32_t flags, hm_export_t *out, hipStream_t s) {
    int rc = check_table(t);
    if (rc) return rc;
    if (!out || !out->n_out) return fail(HM_EINVAL, "export: out or n_out is NULL");
    if (out->capacity > 0 && (!out->key_hi || !out->key_lo || !out->count || !out->tl || !out->tr || !out->cls_l ||
                              !out->cls_r))
        return fail(HM_EINVAL, "export: record arrays are NULL");
    if (flags & ~(HM_EXPORT_UU_ONLY | HM_EXPORT_ALL | HM_EXPORT_CLASSIFY | HM_EXPORT_SORTED))
        return fail(HM_EINVAL, "export: unknown flags");
    if (flags & HM_EXPORT_SORTED) {
        if (out->capacity >= (1ull << 32)) return fail(HM_EINVAL, "export: HM_EXPORT_SORTED needs capacity < 2^32");
        if (out->capacity > 0 && (!out->sort_work || ((uintptr_t)out->sort_work & 255)))
            return fail(HM_EINVAL, "export: HM_EXPORT_SORTED needs a 256-byte aligned sort_work");
        if (out->capacity > 0 && out->sort_work_bytes < sort_work_bytes(out->capacity))
            return fail(HM_EINVAL, "export: sort_work has %llu bytes, %llu needed",
                        (unsigned long long)out->sort_work_bytes,
                        (unsigned long long)sort_work_bytes(out->capacity));
    }
    if ((flags & HM_EXPORT_CLASSIFY) && (out->min_depth < 1 || out->ext_min < 1))
        return fail(HM_EINVAL, "export: HM_EXPORT_CLASSIFY needs min_depth and ext_min >= 1");
    if (out->capacity > 0 && (((uintptr_t)out->tl | (uintptr_t)out->tr) & 15))
        return fail(HM_EINVAL, "export: tl and tr must be 16-byte aligned");
    if (t->k < 1 || t->k > 63) return fail(HM_EINVAL, "table k must be 1..63");
    rc = fill<uint64_t>(out->n_out, 1, 0ull, s);
    if (rc) return rc;
    if (out->digest) {
        rc = fill<uint64_t>(out->digest, 2, 0ull, s);
        if (rc) return rc;
    }
    const dim3 g((unsigned)grid_for(t->capacity, 16));
    uint4 *staged = (flags & HM_EXPORT_SORTED) && out->capacity ? sort_staging(*out) : nullptr;
#define LAUNCH_EXPORT(KW, PER)                                                                              \
    hipLaunchKernelGGL((k_export<KW, PER>), g, dim3(kBlock), 0, s, reinterpret_cast<const Slot *>(t->slots), \
                       t->capacity, flags, *out, t->status, staged)
    if (t->k >= 32) {
        if (staged) LAUNCH_EXPORT(2, kExportPerLane);
        else LAUNCH_EXPORT(2, 32);
    } else {
        if (staged) LAUNCH_EXPORT(1, kExportPerLane);
        else LAUNCH_EXPORT(1, 32);
    }
#undef LAUNCH_EXPORT
    HM_LAUNCH_CHECK("hm_export_table");
    if (flags & HM_EXPORT_SORTED) return sort_export(*out, 2 * t->k, s);
    return HM_OK;
}

}  // extern "C"
