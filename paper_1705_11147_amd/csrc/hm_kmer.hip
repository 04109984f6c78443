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
//   * Slots are 64 bytes (one per cache line): two key words, each carrying a
//     "written" bit so a reader can tell a half-published two-word key from a
//     complete one without fences, then u32 counters: tl[4], tr[4] and nl
//     (occurrences without a left extension); count = nl + sum(tl).
//     A hit therefore costs one atomic add on the left counter and one on the
//     right counter, both on the line the probe already touched.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>

#include "hm_kmer.h"

namespace {

constexpr uint64_t kWritten = 1ull << 63;   // set in every written key word
constexpr uint64_t kLow63 = kWritten - 1;
constexpr uint64_t kOwnerSeed = 0x243F6A8885A308D3ull;  // owner map (definition constant)
constexpr int kBlock = 256;
constexpr int kTileBases = 16384;           // bases staged in LDS per tile
constexpr int kTileMaskWords = kTileBases / 64 + 4;
constexpr int kTileB2Words = 2 * kTileMaskWords;
constexpr int kVarReads = 256;              // reads per tile on the variable-length path
constexpr uint32_t kMaxSpin = 1u << 22;     // bound on re-reads of a half-published slot
constexpr uint32_t kDefaultMaxProbe = 4096; // default linear-probe bound
constexpr uint32_t kAbortBits = HM_ST_TABLE_FULL | HM_ST_LIST_FULL;

// True once a pass has failed (table or list full): the table will be rebuilt
// by the caller, so the remaining work is skipped.  Wave-uniform.
__device__ __forceinline__ bool aborted(const uint32_t *status) {
    const uint32_t st = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (__builtin_amdgcn_readfirstlane(st) & kAbortBits) != 0;
}

struct Slot {
    uint64_t a;       // k <= 31: key | written;  k >= 32: key bits 63..125 | written
    uint64_t b;       // k >= 32: key bits 0..62 | written
    uint32_t tl[4];
    uint32_t tr[4];
    uint32_t nl;      // occurrences with no left extension
    uint32_t cls;     // classify: cls_l | cls_r << 8 | kept << 16 | count >= 2^32 << 17
    uint64_t pad;
};
static_assert(sizeof(Slot) == HM_SLOT_BYTES, "slot is one 64-byte line");

#define RLX __ATOMIC_RELAXED
#define AGT __HIP_MEMORY_SCOPE_AGENT

// ------------------------------------------------------------------ hashing

// 64-bit finalizer of MurmurHash3 (Austin Appleby, public domain).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// table / Bloom hash of a key (any good mixer; the output does not depend on it)
__device__ __forceinline__ uint64_t key_hash(uint64_t hi, uint64_t lo, uint64_t seed) {
    return fmix64(lo ^ fmix64(hi ^ seed));
}

// owner-computes map: floor(H * n / 2^64), H = fmix64(fmix64(hi ^ s) ^ lo)
__device__ __forceinline__ uint32_t owner_of(uint64_t hi, uint64_t lo, uint32_t n) {
    uint64_t h = fmix64(fmix64(hi ^ kOwnerSeed) ^ lo);
    return (uint32_t)__umul64hi(h, (uint64_t)n);
}

// ------------------------------------------------------------------ 2-bit code helpers

// reverse the order of the 32 two-bit groups of a word
__device__ __forceinline__ uint64_t rev2(uint64_t x) {
    x = __builtin_bswap64(x);
    x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
    x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
    return x;
}

struct U128 {
    uint64_t hi, lo;
};

// reverse complement of the 2k-bit code x
__device__ __forceinline__ U128 revcomp(U128 x, int k) {
    const uint64_t nh = rev2(~x.lo), nl = rev2(~x.hi);  // complement + reverse all 128 bits
    const int sh = 128 - 2 * k;
    U128 r;
    if (sh >= 64) {
        r.hi = 0;
        r.lo = nh >> (sh - 64);
    } else {
        r.lo = (nl >> sh) | (nh << (64 - sh));
        r.hi = nh >> sh;
    }
    return r;
}

// Packed words of a tile (LDS) or of the whole batch (global), addressed by a
// base index relative to `org` (a multiple of 64).
struct Words {
    const uint64_t *b2, *nm, *hq;
    __device__ __forceinline__ uint64_t code(int64_t j) const {
        const uint64_t w = b2[j >> 5];
        return (w >> (62 - 2 * (j & 31))) & 3;
    }
    __device__ __forceinline__ bool hqbit(int64_t j) const { return (hq[j >> 6] >> (63 - (j & 63))) & 1; }
    // k validity bits starting at base j are all clear
    __device__ __forceinline__ bool window_valid(int64_t j, int k) const {
        const int64_t i = j >> 6;
        const int s = (int)(j & 63);
        uint64_t m = nm[i] << s;
        if (s) m |= nm[i + 1] >> (64 - s);
        return (m >> (64 - k)) == 0;
    }
    // 2k-bit forward code of the window starting at base j
    __device__ __forceinline__ U128 window(int64_t j, int k) const {
        const int64_t p = 2 * j;
        const int64_t i = p >> 6;
        const int s = (int)(p & 63);
        const uint64_t w0 = b2[i], w1 = b2[i + 1];
        const uint64_t x0 = s ? (w0 << s) | (w1 >> (64 - s)) : w0;
        U128 r;
        if (2 * k <= 64) {
            r.hi = 0;
            r.lo = x0 >> (64 - 2 * k);
        } else {
            const uint64_t w2 = b2[i + 2];
            const uint64_t x1 = s ? (w1 << s) | (w2 >> (64 - s)) : w1;
            const int sh = 128 - 2 * k;
            r.lo = (x1 >> sh) | (x0 << (64 - sh));
            r.hi = x0 >> sh;
        }
        return r;
    }
};

// One k-mer occurrence after extraction.
struct Occ {
    uint64_t hi, lo;  // canonical key
    int left, right;  // extension base 0..3, or 4 = none
};

// Extract the occurrence whose window starts at base j of a read spanning
// [rb, re) (all relative to the Words origin).  Returns false when the window
// holds a non-ACGT base or the key belongs to another owner.
__device__ __forceinline__ bool extract(const Words &w, int64_t j, int64_t rb, int64_t re, int k, bool forward_only,
                                        uint32_t n_owners, uint32_t owner, Occ &o) {
    if (!w.window_valid(j, k)) return false;
    const U128 f = w.window(j, k);
    const bool lok = j > rb && w.hqbit(j - 1);
    const bool rok = j + k < re && w.hqbit(j + k);
    const int lb = lok ? (int)w.code(j - 1) : 4;
    const int rb_ = rok ? (int)w.code(j + k) : 4;
    bool fwd = true;
    U128 r = f;
    if (!forward_only) {
        r = revcomp(f, k);
        fwd = (f.hi < r.hi) || (f.hi == r.hi && f.lo <= r.lo);
    }
    o.hi = fwd ? f.hi : r.hi;
    o.lo = fwd ? f.lo : r.lo;
    o.left = fwd ? lb : (rb_ < 4 ? 3 - rb_ : 4);
    o.right = fwd ? rb_ : (lb < 4 ? 3 - lb : 4);
    if (n_owners > 1 && owner_of(o.hi, o.lo, n_owners) != owner) return false;
    return true;
}

// ------------------------------------------------------------------ table

// slot key words of a canonical key
template <int KW>
__device__ __forceinline__ void slot_words(uint64_t hi, uint64_t lo, uint64_t &A, uint64_t &B) {
    if (KW == 1) {
        A = lo | kWritten;
        B = 0;
    } else {
        A = ((hi << 1) | (lo >> 63)) | kWritten;
        B = (lo & kLow63) | kWritten;
    }
}

// Result of a table probe: slot >= 0 where the key is (or was inserted);
// -1 absent, with `at` the empty slot that ended the probe; -2 probe bound
// reached.  `used` counts the slots probed.
struct Probe {
    int64_t slot;
    uint64_t at;
    uint32_t used;
};

// Locate (A, B) by linear probing from `start` (the first `used0` slots of
// the sequence were already probed by an earlier call).  COHERENT: the table
// is being written by this kernel (device-scope atomic loads); otherwise keys
// are immutable and plain loads suffice.  With `insert`, an absent key claims
// the first empty slot: CAS on word a, then store of word b.  A reader that
// sees a matching a and an unwritten b re-reads the slot.  Key words are
// written once and never cleared, so a probe that stopped at an empty slot
// can resume there.
template <int KW, bool COHERENT>
__device__ __forceinline__ Probe table_find(Slot *slots, uint64_t cmask, uint64_t start, uint64_t A, uint64_t B,
                                            uint32_t max_probe, bool insert, uint32_t used0 = 0) {
    uint64_t i = start & cmask;
    uint32_t probes = used0, spins = 0;
    while (true) {
        Slot *s = slots + i;
        uint64_t a = COHERENT ? __hip_atomic_load(&s->a, RLX, AGT) : s->a;
        if (a == 0) {
            if (!insert) return Probe{-1, i, probes};
            uint64_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(&s->a, &expected, A, RLX, RLX, AGT)) {
                if (KW == 2) __hip_atomic_store(&s->b, B, RLX, AGT);
                return Probe{(int64_t)i, i, probes};
            }
            a = expected;
        }
        if (a == A) {
            if (KW == 1) return Probe{(int64_t)i, i, probes};
            const uint64_t b = COHERENT ? __hip_atomic_load(&s->b, RLX, AGT) : s->b;
            if (b == B) return Probe{(int64_t)i, i, probes};
            // claimed for a key with the same word a, word b not visible yet: re-read
            if (COHERENT && b == 0) {
                if (++spins > kMaxSpin) return Probe{-2, i, probes};
                continue;
            }
        }
        i = (i + 1) & cmask;
        if (++probes >= max_probe) return Probe{-2, i, probes};
    }
}

template <bool CHECKED>
__device__ __forceinline__ void count_occurrence(Slot *s, int left, int right, uint32_t *status) {
    uint32_t *lp = left < 4 ? &s->tl[left] : &s->nl;
    if (CHECKED) {
        uint32_t o = __hip_atomic_fetch_add(lp, 1u, RLX, AGT);
        uint32_t o2 = right < 4 ? __hip_atomic_fetch_add(&s->tr[right], 1u, RLX, AGT) : 0u;
        if (o == 0xFFFFFFFFu || o2 == 0xFFFFFFFFu) atomicOr(status, HM_ST_OVERFLOW);
    } else {
        __hip_atomic_fetch_add(lp, 1u, RLX, AGT);
        if (right < 4) __hip_atomic_fetch_add(&s->tr[right], 1u, RLX, AGT);
    }
}

// ------------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ------------------------------------------------------------------ kernels

struct PassArgs {
    const uint64_t *b2, *nm, *hq;
    const int64_t *read_off;
    int64_t n_reads;
    int64_t n_bases;
    int32_t read_len;
    int32_t k;
    uint32_t forward_only;
    uint32_t n_owners, owner;
    uint64_t seed;
    // bloom
    uint64_t *bloom;
    uint64_t bloom_mask;  // n_words - 1
    uint32_t n_hash;
    uint32_t bypass;
    // table
    Slot *slots;
    uint64_t cmask;
    uint32_t max_probe;
    uint32_t *status;
    unsigned long long *stats;  // optional event counters (hm_table_t.stats)
    // first-occurrence list
    uint64_t *lkeys;
    uint8_t *lext;
    uint64_t lcap;
    unsigned long long *lcount;
};

// Per-lane event counts of a counting pass (see HM_STAT_* in hm_kmer.h).
struct Stats {
    uint32_t v[HM_N_STATS];
};

// Sum a wave's counts and add them to the table's counters (one atomic per
// counter per wave).
__device__ __forceinline__ void stats_flush(unsigned long long *dst, const Stats &st) {
    if (!dst) return;
#pragma unroll
    for (int i = 0; i < HM_N_STATS; ++i) {
        uint64_t x = st.v[i];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane_id() == 0 && x) atomicAdd(dst + i, (unsigned long long)x);
    }
}

// Per-wave cursor into the first-occurrence list.  A wave reserves
// kListChunk entries at a time with one atomic add, so the shared counter sees
// one atomic per chunk instead of one per wave iteration.  Entries of a chunk
// the wave leaves unused are marked as holes (ext = kHole) at kernel end.
constexpr uint32_t kListChunk = 256;
constexpr uint8_t kHole = 0xFF;

struct ListCursor {
    uint64_t base;  // first entry of the current chunk
    uint32_t used;  // entries of the chunk handed out (kListChunk: no chunk yet)
};

// Per-occurrence body of pass 1.  `act` lanes carry an occurrence; every lane
// of the wave must call it (list appends are aggregated per wave).
template <int KW, bool CHECKED>
__device__ __forceinline__ void pass1_occ(const PassArgs &a, bool act, const Occ &o, ListCursor &cur, Stats &st) {
    // The table is probed first: an occurrence whose k-mer is already there is
    // counted without touching the Bloom filter.  Only absent k-mers test and
    // set their Bloom bits; a k-mer the filter has seen is inserted and this
    // occurrence counted, an unseen one goes to the first-occurrence list.
    bool deferred = false;
    if (act) {
        const uint64_t h = key_hash(o.hi, o.lo, a.seed);
        uint64_t A, B;
        slot_words<KW>(o.hi, o.lo, A, B);
        Probe pr = table_find<KW, true>(a.slots, a.cmask, h, A, B, a.max_probe, a.bypass != 0);
        st.v[HM_STAT_OCC] += 1;
        st.v[HM_STAT_HIT] += pr.slot >= 0 ? 1u : 0u;
        if (pr.slot == -1) {
            st.v[HM_STAT_BLOOM] += 1;
            const uint64_t g = fmix64(h + 0x9E3779B97F4A7C15ull);
            uint64_t mask = 0;
            for (uint32_t j = 0; j < a.n_hash; ++j) mask |= 1ull << ((g >> (6 * j)) & 63);
            uint64_t *w = a.bloom + ((h >> 24) & a.bloom_mask);
            const uint64_t old = __hip_atomic_fetch_or(w, mask, RLX, AGT);
            if ((old & mask) == mask) pr = table_find<KW, true>(a.slots, a.cmask, pr.at, A, B, a.max_probe, true, pr.used);
            else deferred = true;
        }
        st.v[HM_STAT_DEFER] += deferred ? 1u : 0u;
        st.v[HM_STAT_PROBES] += pr.used + 1;
        if (pr.slot >= 0) count_occurrence<CHECKED>(a.slots + pr.slot, o.left, o.right, a.status);
        else if (pr.slot == -2) atomicOr(a.status, HM_ST_TABLE_FULL);
    }
    if (!a.bypass) {
        const bool need = deferred;
        const uint64_t m = __ballot(need);
        if (m) {
            const uint32_t n = (uint32_t)__popcll(m);
            const uint32_t pos = cur.used + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1));
            uint64_t fresh = 0;
            if (cur.used + n > kListChunk) {  // wave-uniform: take a new chunk
                const int leader = __ffsll((long long)m) - 1;
                if ((int)lane_id() == leader) fresh = atomicAdd(a.lcount, (unsigned long long)kListChunk);
                fresh = __shfl(fresh, leader);
            }
            if (need) {
                const uint64_t idx = pos < kListChunk ? cur.base + pos : fresh + (pos - kListChunk);
                if (idx < a.lcap) {
                    a.lkeys[2 * idx] = o.hi;
                    a.lkeys[2 * idx + 1] = o.lo;
                    a.lext[idx] = (uint8_t)(o.left | (o.right << 4));
                } else {
                    atomicOr(a.status, HM_ST_LIST_FULL);
                }
            }
            cur.used += n;
            if (cur.used > kListChunk) {
                cur.base = fresh;
                cur.used -= kListChunk;
            }
        }
    }
}

// Mark the unused tail of the wave's current chunk as holes.
__device__ __forceinline__ void list_close(const PassArgs &a, const ListCursor &cur) {
    if (a.bypass || cur.used >= kListChunk) return;
    for (uint32_t i = cur.used + lane_id(); i < kListChunk; i += 64) {
        const uint64_t idx = cur.base + i;
        if (idx < a.lcap) a.lext[idx] = kHole;
    }
}

// Pass 1 over fixed-length reads: tiles of whole reads staged in LDS.
template <int KW, bool CHECKED>
__global__ __launch_bounds__(kBlock) void k_pass1_fixed(PassArgs a, int32_t reads_per_tile, int64_t n_tiles) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    const int L = a.read_len;
    const int k = a.k;
    const int W = L - k + 1;  // windows per read (> 0, checked by the host)
    ListCursor cur{0, kListChunk};
    Stats st = {};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t base0 = r0 * L, base1 = r1 * L;
        const int64_t org = base0 & ~(int64_t)63;          // origin: multiple of 64 bases
        const int64_t mw0 = org >> 6;
        const int nmw = (int)(((base1 + 63) >> 6) - mw0) + 2;  // mask words incl. 2 guard words
        __syncthreads();  // previous tile's readers are done
        for (int i = threadIdx.x; i < nmw; i += kBlock) {
            s_nm[i] = a.nm[mw0 + i];
            s_hq[i] = a.hq[mw0 + i];
        }
        for (int i = threadIdx.x; i < 2 * nmw; i += kBlock) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        const Words w{s_b2, s_nm, s_hq};
        const int total = (int)(r1 - r0) * W;
        for (int f0 = 0; f0 < total; f0 += kBlock) {
            if (aborted(a.status)) break;
            const int f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            if (f < total) {
                const int r = f / W;
                const int pos = f - r * W;
                const int64_t rb = (r0 + r) * L - org;
                act = extract(w, rb + pos, rb, rb + L, k, a.forward_only, a.n_owners, a.owner, o);
            }
            pass1_occ<KW, CHECKED>(a, act, o, cur, st);
        }
    }
    list_close(a, cur);
    stats_flush(a.stats, st);
}

// Pass 1 over variable-length reads (read_off given): packed words are read
// from global memory; a per-tile prefix sum in LDS maps flat window indices
// to reads.
template <int KW, bool CHECKED>
__global__ __launch_bounds__(kBlock) void k_pass1_var(PassArgs a, int64_t n_tiles) {
    __shared__ int64_t s_off[kVarReads + 1];
    __shared__ int64_t s_pre[kVarReads + 1];
    const int k = a.k;
    const Words w{a.b2, a.nm, a.hq};
    ListCursor cur{0, kListChunk};
    Stats st = {};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * kVarReads;
        const int nr = (int)min((int64_t)kVarReads, a.n_reads - r0);
        __syncthreads();
        // offsets clamped to [0, n_bases]; a decreasing offset makes an empty read
        for (int i = threadIdx.x; i <= nr; i += kBlock) s_off[i] = min(max(a.read_off[r0 + i], (int64_t)0), a.n_bases);
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t acc = 0;
            for (int i = 0; i < nr; ++i) {
                s_pre[i] = acc;
                const int64_t len = s_off[i + 1] - s_off[i];
                acc += len >= k ? len - k + 1 : 0;
            }
            s_pre[nr] = acc;
        }
        __syncthreads();
        const int64_t total = s_pre[nr];
        for (int64_t f0 = 0; f0 < total; f0 += kBlock) {
            if (aborted(a.status)) break;
            const int64_t f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            if (f < total) {
                int lo = 0, hi = nr;  // last read r with s_pre[r] <= f
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= f) lo = mid;
                    else hi = mid;
                }
                const int64_t rb = s_off[lo], re = max(s_off[lo + 1], rb);
                act = extract(w, rb + (f - s_pre[lo]), rb, re, k, a.forward_only, a.n_owners, a.owner, o);
            }
            pass1_occ<KW, CHECKED>(a, act, o, cur, st);
        }
    }
    list_close(a, cur);
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
        const uint64_t hi = a.lkeys[2 * i], lo = a.lkeys[2 * i + 1];
        const uint8_t e = a.lext[i];
        if (e == kHole) continue;
        uint64_t A, B;
        slot_words<KW>(hi, lo, A, B);
        const Probe pr = table_find<KW, false>(a.slots, a.cmask, key_hash(hi, lo, a.seed), A, B, a.max_probe, false);
        st.v[HM_STAT_P2_ENTRIES] += 1;
        st.v[HM_STAT_P2_FOUND] += pr.slot >= 0 ? 1u : 0u;
        if (pr.slot >= 0) count_occurrence<CHECKED>(a.slots + pr.slot, e & 15, e >> 4, a.status);
        else if (pr.slot == -2) atomicOr(a.status, HM_ST_TABLE_FULL);
    }
    stats_flush(a.stats, st);
}

__device__ __forceinline__ uint32_t side_class(const uint32_t t[4], uint32_t ext_min) {
    uint32_t n = 0, b = 0;
    for (uint32_t i = 0; i < 4; ++i)
        if (t[i] >= ext_min) {
            ++n;
            b = i;
        }
    return n == 0 ? (uint32_t)HM_CLS_X : (n == 1 ? b : (uint32_t)HM_CLS_FORK);
}

__global__ __launch_bounds__(kBlock) void k_classify(Slot *slots, uint64_t cap, uint32_t min_depth, uint32_t ext_min) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * kBlock) {
        Slot *s = slots + i;
        if (s->a == 0) continue;
        uint32_t tl[4], tr[4];
        for (int b = 0; b < 4; ++b) {
            tl[b] = s->tl[b];
            tr[b] = s->tr[b];
        }
        const uint64_t cnt = (uint64_t)s->nl + tl[0] + tl[1] + tl[2] + tl[3];
        const uint32_t kept = cnt >= min_depth ? 1u : 0u;
        const uint32_t ovf = cnt > 0xFFFFFFFFull ? 1u : 0u;
        s->cls = side_class(tl, ext_min) | (side_class(tr, ext_min) << 8) | (kept << 16) | (ovf << 17);
    }
}

__device__ __forceinline__ uint64_t record_hash(uint64_t hi, uint64_t lo, uint32_t cnt, const uint32_t tl[4],
                                                const uint32_t tr[4], uint32_t cl, uint32_t cr) {
    uint64_t x = fmix64(hi ^ 0x6A09E667F3BCC908ull);
    x = fmix64(x ^ lo);
    x = fmix64(x ^ cnt);
    for (int b = 0; b < 4; ++b) x = fmix64(x ^ (((uint64_t)tl[b] << 32) | tr[b]));
    return fmix64(x ^ (cl | (cr << 8)));
}

constexpr int kExportPerLane = 8;

template <int KW>
__global__ __launch_bounds__(kBlock) void k_export(const Slot *slots, uint64_t cap, uint32_t flags, hm_export_t out,
                                                   uint32_t *status) {
    uint64_t dsum = 0, dxor = 0;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * kBlock) >> 6;
    const uint64_t per_iter = 64 * kExportPerLane;  // slots per wave iteration
    const uint64_t iters = (cap + per_iter * n_waves - 1) / (per_iter * n_waves);
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t first = (it * n_waves + wave) * per_iter;
        // pass A: which of this lane's slots are taken (slots first + j*64 + lane, coalesced per j)
        uint32_t take_bits = 0;
#pragma unroll
        for (int j = 0; j < kExportPerLane; ++j) {
            const uint64_t i = first + (uint64_t)j * 64 + lane;
            if (i < cap) {
                const Slot *sl = slots + i;
                if (sl->a != 0) {
                    const uint32_t c = sl->cls;
                    const bool kept = (c >> 16) & 1;
                    bool take = (flags & HM_EXPORT_ALL) ? true : kept;
                    if (flags & HM_EXPORT_UU_ONLY) take = take && kept && (c & 0xFF) < 4 && ((c >> 8) & 0xFF) < 4;
                    if ((c >> 17) & 1) atomicOr(status, HM_ST_OVERFLOW);
                    take_bits |= (take ? 1u : 0u) << j;
                }
            }
        }
        // wave-wide exclusive prefix of the per-lane counts, one atomic per wave
        const uint32_t cnt = (uint32_t)__popc(take_bits);
        uint32_t incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d);
            if ((int)lane >= d) incl += y;
        }
        const uint32_t total = __shfl(incl, 63);
        if (total == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_out), (unsigned long long)total);
        base = __shfl(base, 0);
        uint64_t idx = base + (incl - cnt);
        // pass B: write this lane's records
#pragma unroll
        for (int j = 0; j < kExportPerLane; ++j) {
            if (!((take_bits >> j) & 1)) continue;
            const Slot *sl = slots + first + (uint64_t)j * 64 + lane;
            uint64_t hi = 0, lo;
            if (KW == 1) {
                lo = sl->a & kLow63;
            } else {
                const uint64_t A = sl->a & kLow63, B = sl->b & kLow63;
                lo = B | (A << 63);
                hi = A >> 1;
            }
            uint32_t tl[4], tr[4];
            for (int b = 0; b < 4; ++b) {
                tl[b] = sl->tl[b];
                tr[b] = sl->tr[b];
            }
            const uint32_t c = sl->cls;
            const uint32_t cl = c & 0xFF, cr = (c >> 8) & 0xFF;
            const uint32_t count = sl->nl + tl[0] + tl[1] + tl[2] + tl[3];
            if (idx < out.capacity) {
                out.key_hi[idx] = hi;
                out.key_lo[idx] = lo;
                out.count[idx] = count;
                for (int b = 0; b < 4; ++b) {
                    out.tl[4 * idx + b] = tl[b];
                    out.tr[4 * idx + b] = tr[b];
                }
                out.cls_l[idx] = (uint8_t)cl;
                out.cls_r[idx] = (uint8_t)cr;
            } else {
                atomicOr(status, HM_ST_OUTPUT_FULL);
            }
            if (out.digest) {
                const uint64_t x = record_hash(hi, lo, count, tl, tr, cl, cr);
                dsum += x;
                dxor ^= x;
            }
            ++idx;
        }
    }
    if (out.digest) {
        for (int off = 32; off > 0; off >>= 1) {
            dsum += __shfl_xor(dsum, off);
            dxor ^= __shfl_xor(dxor, off);
        }
        if (lane == 0 && (dsum | dxor)) {
            atomicAdd(reinterpret_cast<unsigned long long *>(out.digest), (unsigned long long)dsum);
            atomicXor(reinterpret_cast<unsigned long long *>(out.digest + 1), (unsigned long long)dxor);
        }
    }
}

// ASCII + Phred -> 2-bit codes and masks; one thread per 64 bases (one mask word).
__device__ __forceinline__ void pack16(uint4 sa, uint4 sq, int nvalid, int qual_offset, int qcut, uint64_t &codes,
                                       uint32_t &bad, uint32_t &good) {
    // codes: 16 bases x 2 bits, first base most significant; bad/good: 16 bits, first base most significant
    const uint32_t av[4] = {sa.x, sa.y, sa.z, sa.w};
    const uint32_t qv[4] = {sq.x, sq.y, sq.z, sq.w};
    codes = 0;
    bad = 0;
    good = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t x = ((av[i >> 2] >> (8 * (i & 3))) & 0xFFu) | 0x20u;  // fold case
        const int q = (int)((qv[i >> 2] >> (8 * (i & 3))) & 0xFFu);
        const uint32_t code = (x == 'c') ? 1u : (x == 'g') ? 2u : (x == 't') ? 3u : 0u;
        const bool valid = i < nvalid && ((x == 'a') | (x == 'c') | (x == 'g') | (x == 't'));
        codes = (codes << 2) | (valid ? code : 0u);
        bad = (bad << 1) | (valid ? 0u : 1u);
        good = (good << 1) | ((valid && q - qual_offset >= qcut) ? 1u : 0u);
    }
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, uint64_t n, T v) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) p[i] = v;
}

// ------------------------------------------------------------------ host side

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(HM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HM_LAUNCH_CHECK(what)                           \
    do {                                                \
        hipError_t e_ = hipGetLastError();              \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

std::atomic<int> g_cus[64];

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

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

uint64_t grid_for(uint64_t items, int per_cu = 8) {
    const uint64_t blocks = (items + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)device_cus() * per_cu;
    return blocks < 1 ? 1 : (blocks < cap ? blocks : cap);
}

template <typename T>
int fill(T *p, uint64_t n, T v, hipStream_t s) {
    if (n == 0) return HM_OK;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)grid_for(n, 16)), dim3(kBlock), 0, s, p, n, v);
    HM_LAUNCH_CHECK("fill");
    return HM_OK;
}

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

int check_table(const hm_table_t *t) {
    if (!t || !t->slots || !t->status) return fail(HM_EINVAL, "table or its buffers are NULL");
    if (!pow2(t->capacity)) return fail(HM_EINVAL, "table capacity must be a power of two");
    if (((uintptr_t)t->slots) & 63) return fail(HM_EINVAL, "table slots must be 64-byte aligned");
    return HM_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

int hm_abi_version(void) { return HM_ABI_VERSION; }

const char *hm_last_error(void) { return g_err; }

uint64_t hm_mask_words(int64_t n_bases) { return (uint64_t)(n_bases < 0 ? 0 : n_bases) / 64 + 3; }

uint64_t hm_bases2_words(int64_t n_bases) { return 2 * hm_mask_words(n_bases); }

size_t hm_table_bytes(uint64_t capacity) { return (size_t)capacity * HM_SLOT_BYTES; }

size_t hm_bloom_bytes(uint64_t n_words) { return (size_t)n_words * 8; }

size_t hm_list_bytes(uint64_t capacity) { return (size_t)capacity * 17; }

int hm_check_params(const hm_params_t *p) {
    if (!p) return fail(HM_EINVAL, "params is NULL");
    if (p->k < 1 || p->k > 63) return fail(HM_EINVAL, "k must be in 1..63 (got %d)", p->k);
    if (!(p->flags & HM_FORWARD_ONLY) && (p->k % 2) == 0)
        return fail(HM_EINVAL, "k must be odd for canonical k-mers (got %d)", p->k);
    if (p->min_depth < 1) return fail(HM_EINVAL, "min_depth must be >= 1");
    if (p->ext_min < 1) return fail(HM_EINVAL, "ext_min must be >= 1");
    if (p->n_owners < 1 || p->owner >= p->n_owners) return fail(HM_EINVAL, "owner must be < n_owners");
    if (p->flags & ~(HM_FORWARD_ONLY | HM_BLOOM_BYPASS | HM_CHECKED)) return fail(HM_EINVAL, "unknown flags");
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
    return fill<uint64_t>(l->count, 1, 0ull, s);
}

int hm_status(const hm_table_t *t, hipStream_t s) {
    if (!t || !t->status) return fail(HM_EINVAL, "table status is NULL");
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t st = 0;
    e = hipMemcpy(&st, t->status, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status)");
    if (st & HM_ST_OVERFLOW) return fail(HM_EOVERFLOW, "a k-mer counter passed 2^32 - 1 (status 0x%x)", st);
    if (st & (HM_ST_TABLE_FULL | HM_ST_LIST_FULL))
        return fail(HM_ECAPACITY, "%s full (status 0x%x)", (st & HM_ST_TABLE_FULL) ? "count table" : "first-occurrence list",
                    st);
    if (st & HM_ST_OUTPUT_FULL) return fail(HM_EOUTPUT, "export buffer too small (status 0x%x)", st);
    return HM_OK;
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
        if (!b || !b->words || !pow2(b->n_words) || b->n_hash < 1 || b->n_hash > 8)
            return fail(HM_EINVAL, "a Bloom filter (power-of-two words, 1..8 hashes) is needed unless bypassed");
        if (b->n_words > (1ull << 40)) return fail(HM_EINVAL, "bloom too large");
        a.bloom = b->words;
        a.bloom_mask = b->n_words - 1;
        a.n_hash = b->n_hash;
    }
    if (!bypass || !need_reads) {
        if (!l || !l->keys || !l->ext || !l->count) return fail(HM_EINVAL, "first-occurrence list is NULL");
        a.lkeys = l->keys;
        a.lext = l->ext;
        a.lcap = l->capacity;
        a.lcount = reinterpret_cast<unsigned long long *>(l->count);
    }
    a.slots = reinterpret_cast<Slot *>(t->slots);
    a.cmask = t->capacity - 1;
    const uint64_t mp = t->max_probe ? (uint64_t)t->max_probe : (uint64_t)kDefaultMaxProbe;
    a.max_probe = (uint32_t)(mp < t->capacity ? mp : t->capacity);
    a.status = t->status;
    a.stats = reinterpret_cast<unsigned long long *>(t->stats);
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
    const int grid_cap = device_cus() * 8;
    if (!r->read_off && r->read_len <= kTileBases - 64) {
        if (r->read_len < p->k) return HM_OK;  // no windows
        const int32_t rpt = kTileBases / r->read_len;
        const int64_t n_tiles = (r->n_reads + rpt - 1) / rpt;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
#define LAUNCH_FIXED(KW, CH) hipLaunchKernelGGL((k_pass1_fixed<KW, CH>), g, dim3(kBlock), 0, s, a, rpt, n_tiles)
        if (two) { if (checked) LAUNCH_FIXED(2, true); else LAUNCH_FIXED(2, false); }
        else { if (checked) LAUNCH_FIXED(1, true); else LAUNCH_FIXED(1, false); }
#undef LAUNCH_FIXED
    } else {
        if (!r->read_off) return fail(HM_EINVAL, "reads longer than %d bases need read_off", kTileBases - 64);
        const int64_t n_tiles = (r->n_reads + kVarReads - 1) / kVarReads;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
#define LAUNCH_VAR(KW, CH) hipLaunchKernelGGL((k_pass1_var<KW, CH>), g, dim3(kBlock), 0, s, a, n_tiles)
        if (two) { if (checked) LAUNCH_VAR(2, true); else LAUNCH_VAR(2, false); }
        else { if (checked) LAUNCH_VAR(1, true); else LAUNCH_VAR(1, false); }
#undef LAUNCH_VAR
    }
    HM_LAUNCH_CHECK("hm_bloom_insert");
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
                       reinterpret_cast<Slot *>(t->slots), t->capacity, p->min_depth, p->ext_min);
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
    if (flags & ~(HM_EXPORT_UU_ONLY | HM_EXPORT_ALL)) return fail(HM_EINVAL, "export: unknown flags");
    if (t->k < 1 || t->k > 63) return fail(HM_EINVAL, "table k must be 1..63");
    rc = fill<uint64_t>(out->n_out, 1, 0ull, s);
    if (rc) return rc;
    if (out->digest) {
        rc = fill<uint64_t>(out->digest, 2, 0ull, s);
        if (rc) return rc;
    }
    const dim3 g((unsigned)grid_for(t->capacity, 16));
    if (t->k >= 32)
        hipLaunchKernelGGL(k_export<2>, g, dim3(kBlock), 0, s, reinterpret_cast<const Slot *>(t->slots), t->capacity,
                           flags, *out, t->status);
    else
        hipLaunchKernelGGL(k_export<1>, g, dim3(kBlock), 0, s, reinterpret_cast<const Slot *>(t->slots), t->capacity,
                           flags, *out, t->status);
    HM_LAUNCH_CHECK("hm_export_table");
    return HM_OK;
}

}  // extern "C"
