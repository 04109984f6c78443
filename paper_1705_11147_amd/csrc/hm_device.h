// Device building blocks shared by the plain and the batched k-mer analysis
// kernels (private to the library; the public interface is include/hm_kmer.h).
#pragma once

#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>

#include "hm_kmer.h"

namespace hm {


constexpr uint64_t kWritten = 1ull << 63;   // set in every written key word
constexpr uint64_t kLow63 = kWritten - 1;
constexpr uint64_t kWideBit = 1ull << 63;   // narrow counters frozen, counting goes wide
constexpr int kCasTries = 3;                // narrow CAS attempts before going wide
constexpr uint64_t kOwnerMul1 = 0x9E3779B97F4A7C15ull;  // owner map (definition constants)
constexpr uint64_t kOwnerMul2 = 0xD1B54A32D192ED03ull;
constexpr int kBlock = 256;
constexpr int kTileBases = 16384;           // bases staged in LDS per tile
constexpr int kTileMaskWords = kTileBases / 64 + 4;
constexpr int kTileB2Words = 2 * kTileMaskWords;
constexpr int kVarReads = 256;              // reads per tile on the variable-length path
constexpr uint32_t kMaxSpin = 1u << 22;     // bound on re-reads of a half-published slot
constexpr uint32_t kDefaultMaxProbe = 4096; // default linear-probe bound
constexpr uint32_t kAbortBits = HM_ST_TABLE_FULL | HM_ST_LIST_FULL | HM_ST_STREAM_FULL;

// True once a pass has failed (table or list full): the table will be rebuilt
// by the caller, so the remaining work is skipped.  Wave-uniform.
__device__ __forceinline__ bool aborted(const uint32_t *status) {
    const uint32_t st = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (__builtin_amdgcn_readfirstlane(st) & kAbortBits) != 0;
}

// A slot's counters live in two forms.  `narrow` packs nine 7-bit counters
// (lane 0: occurrences without a left extension, lanes 1..4: left tallies
// A,C,G,T, lanes 5..8: right tallies) and takes one CAS per occurrence.  A
// counter about to pass 127, or repeated CAS contention, sets kWideBit: the
// narrow lanes freeze and later occurrences of the k-mer go to the 32-bit
// wide counters (two atomic adds).  Every occurrence lands in exactly one of
// the two, so the totals are narrow + wide.
struct Slot {
    uint64_t a;       // k <= 31: key | written;  k >= 32: key bits 63..125 | written
    uint64_t narrow;  // 9 x 7-bit counters | kWideBit (next to a: one 16-byte load reads both)
    uint64_t b;       // k >= 32: key bits 0..62 | written
    uint32_t nl;      // wide: occurrences with no left extension
    uint32_t tl[4];   // wide: left tallies
    uint32_t tr[4];   // wide: right tallies
    uint32_t cls;     // classify: cls_l | cls_r << 8 | kept << 16 | count >= 2^32 << 17; while
                      // counting with the filter in the table: Bloom bits of the keys homed here
};
static_assert(sizeof(Slot) == HM_SLOT_BYTES, "slot is one 64-byte line");

#define RLX __ATOMIC_RELAXED
// Eight waves per SIMD (at most 64 registers a lane).  The random-access
// kernels are bound by the memory requests they keep in flight, so spilling a
// few registers to scratch costs less than losing one wave in eight.
#define HM_EIGHT_WAVES __attribute__((amdgpu_waves_per_eu(8, 8)))
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

// owner-computes map: floor(H * n / 2^64), H = (lo ^ hi * m1) * m2 mod 2^64 (multiply-shift:
// the top bits of the product depend on every bit of its operand); for n = 2^b that is the top b
// bits of H (no 64-bit product).  Every window of every read is tested, so the map is kept to two
// 64-bit products.
__device__ __forceinline__ uint32_t owner_of(uint64_t hi, uint64_t lo, uint32_t n) {
    const uint64_t h = (lo ^ hi * kOwnerMul1) * kOwnerMul2;
    if (n <= 1) return 0;
    if ((n & (n - 1)) == 0) return (uint32_t)(h >> (64 - (31 - __clz((int)n))));
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
    uint64_t narrow;  // the slot's narrow counter word as loaded with the key (a hint for the CAS)
    bool inserted;    // this call claimed the slot for the key
};

// Slot of step t of the probe sequence from home slot h: the home slot, the
// other slot of its 128-byte line (which the first access already brought in),
// then the following lines' slots in order.  Every slot appears once.
__device__ __forceinline__ uint64_t probe_slot(uint64_t h, uint32_t t, uint64_t cmask) {
    if (t == 0) return h;
    if (t == 1) return (h ^ 1) & cmask;
    return ((h & ~1ull) + t) & cmask;
}

// Locate (A, B) along the probe sequence from the home slot `start & cmask`
// (the first `used0` slots of the sequence were already probed by an earlier
// call).  With `insert`, an
// absent key claims the first empty slot: CAS on word a, then store of word b;
// a reader that sees a matching a and an unwritten b re-reads b with a
// device-scope atomic load until it is published.  Key words are written once
// and never cleared, so a probe that stopped at an empty slot can resume
// there.
//
// Probes read a and the narrow counter word with one plain 16-byte load (and
// b only when a matches).  A plain load may return an older value of the line
// than another CU's latest atomic, and that is harmless here: a key word is
// either 0 or final, so a stale read can only show a slot as empty.  An
// inserting probe then learns the truth from its CAS; a non-inserting probe
// reports the key absent, and the caller's Bloom test (an atomic) either
// sends it to the inserting probe or defers the occurrence to pass 2, which
// counts it if the key is in the table.  A stale narrow word only makes the
// counting CAS fail once and retry with the value the CAS returned.
template <int KW>
__device__ __forceinline__ Probe table_find(Slot *slots, uint64_t cmask, uint64_t start, uint64_t A, uint64_t B,
                                            uint32_t max_probe, bool insert, uint32_t used0 = 0) {
    const uint64_t home = start & cmask;
    uint32_t probes = used0, spins = 0;
    while (true) {
        const uint64_t i = probe_slot(home, probes, cmask);
        Slot *s = slots + i;
        const uint4 v = *reinterpret_cast<const uint4 *>(s);  // a, narrow
        uint64_t a = (uint64_t)v.x | ((uint64_t)v.y << 32);
        const uint64_t nw = (uint64_t)v.z | ((uint64_t)v.w << 32);
        if (a == 0) {
            if (!insert) return Probe{-1, i, probes, 0, false};
            uint64_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(&s->a, &expected, A, RLX, RLX, AGT)) {
                if (KW == 2) __hip_atomic_store(&s->b, B, RLX, AGT);
                return Probe{(int64_t)i, i, probes, 0, true};
            }
            a = expected;
        }
        if (a == A) {
            if (KW == 1) return Probe{(int64_t)i, i, probes, nw, false};
            uint64_t b = s->b;
            while (b == 0) {  // claimed for a key with the same word a, word b not visible yet
                if (++spins > kMaxSpin) return Probe{-2, i, probes, 0, false};
                b = __hip_atomic_load(&s->b, RLX, AGT);
            }
            if (b == B) return Probe{(int64_t)i, i, probes, nw, false};
        }
        if (++probes >= max_probe) return Probe{-2, i, probes, 0, false};
    }
}

// Count one occurrence with its extensions (left/right: base 0..3 or 4 = none).
// One CAS on the narrow word in the common case; wide 32-bit counters once the
// narrow lanes are frozen.  Returns the number of CAS attempts (for stats).
template <bool CHECKED>
__device__ __forceinline__ uint32_t count_occurrence(Slot *s, int left, int right, uint32_t *status, uint64_t hint) {
    const int ll = left < 4 ? 1 + left : 0;
    const int rl = 5 + right;  // only used when right < 4
    const uint64_t inc = (1ull << (7 * ll)) + (right < 4 ? (1ull << (7 * rl)) : 0ull);
    uint64_t old = hint;
    uint32_t tries = 0;
    while (!(old & kWideBit) && tries < (uint32_t)kCasTries) {
        if (((old >> (7 * ll)) & 127) == 127 || (right < 4 && ((old >> (7 * rl)) & 127) == 127)) break;
        ++tries;
        if (__hip_atomic_compare_exchange_strong(&s->narrow, &old, old + inc, RLX, RLX, AGT)) return tries;
    }
    if (!(old & kWideBit)) __hip_atomic_fetch_or(&s->narrow, kWideBit, RLX, AGT);  // freeze the narrow lanes
    uint32_t *lp = left < 4 ? &s->tl[left] : &s->nl;
    if (CHECKED) {
        uint32_t o = __hip_atomic_fetch_add(lp, 1u, RLX, AGT);
        uint32_t o2 = right < 4 ? __hip_atomic_fetch_add(&s->tr[right], 1u, RLX, AGT) : 0u;
        if (o == 0xFFFFFFFFu || o2 == 0xFFFFFFFFu) atomicOr(status, HM_ST_OVERFLOW);
    } else {
        __hip_atomic_fetch_add(lp, 1u, RLX, AGT);
        if (right < 4) __hip_atomic_fetch_add(&s->tr[right], 1u, RLX, AGT);
    }
    return tries + 16;  // >= 16 marks a wide update
}

// Totals of a slot (narrow + wide), for classification and export.
__device__ __forceinline__ uint64_t slot_counts(const Slot *s, uint32_t tl[4], uint32_t tr[4]) {
    const uint64_t nw = s->narrow;
    uint64_t cnt = (uint64_t)s->nl + (nw & 127);
    for (int b = 0; b < 4; ++b) {
        tl[b] = s->tl[b] + (uint32_t)((nw >> (7 * (1 + b))) & 127);
        tr[b] = s->tr[b] + (uint32_t)((nw >> (7 * (5 + b))) & 127);
        cnt += tl[b];
    }
    return cnt;
}

// ------------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// set bits of the 64-lane mask m below the calling lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

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
    // bloom (nullptr: the filter is in the table's classification words)
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
    // presence filter of the keys pass 1 inserted (optional)
    uint64_t *present;
    uint64_t present_mask;
    uint32_t present_hash;
    // heavy hitters of the table (hm_table_t.heavy), counted per workgroup
    const uint64_t *heavy;
    uint32_t n_heavy;
};

// Word index and bit mask of a key in the presence filter (bits independent
// of the table slot and of the Bloom word).
__device__ __forceinline__ void present_bits(uint64_t h, uint64_t pmask, uint32_t nh, uint64_t &w, uint64_t &m) {
    const uint64_t g = fmix64(h ^ 0xC2B2AE3D27D4EB4Full);
    w = (g >> 40) & pmask;
    m = 0;
    for (uint32_t j = 0; j < nh; ++j) m |= 1ull << ((g >> (6 * j)) & 63);
}

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

// ------------------------------------------------------------------ heavy hitters

// Workgroup-local counters of the table's heavy keys, in dynamic LDS: the
// keys (2 words each), nine counters per key (no left extension, left A..T,
// right A..T) and an open-addressing index of key positions at most half full.
struct HeavyLds {
    uint64_t *keys;
    uint32_t *cnt;
    uint32_t *index;
    uint32_t imask;
    uint32_t n;
};
constexpr uint32_t kNoHeavy = 0xFFFFFFFFu;

__host__ __device__ inline uint32_t heavy_index_size(uint32_t n) {
    uint32_t s = 4;
    while (s < 2 * n) s <<= 1;
    return s;
}

// Dynamic LDS bytes of a pass-1 workgroup for n heavy keys.
__host__ __device__ inline size_t heavy_lds_bytes(uint32_t n) {
    return n ? (size_t)n * (16 + 36) + 4 * (size_t)heavy_index_size(n) : 0;
}

// Load the heavy keys into LDS, clear their counters and build the index.
// Called by every thread of the workgroup (contains barriers).
__device__ __forceinline__ HeavyLds heavy_setup(const PassArgs &a, uint64_t *smem) {
    HeavyLds hv;
    hv.n = a.n_heavy;
    hv.keys = smem;
    hv.cnt = reinterpret_cast<uint32_t *>(smem + 2 * hv.n);
    hv.index = hv.cnt + 9 * hv.n;
    const uint32_t isz = heavy_index_size(hv.n);
    hv.imask = isz - 1;
    for (uint32_t i = threadIdx.x; i < 2 * hv.n; i += kBlock) hv.keys[i] = a.heavy[i];
    for (uint32_t i = threadIdx.x; i < 9 * hv.n; i += kBlock) hv.cnt[i] = 0;
    for (uint32_t i = threadIdx.x; i < isz; i += kBlock) hv.index[i] = kNoHeavy;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < hv.n; e += kBlock) {
        uint32_t i = (uint32_t)(key_hash(hv.keys[2 * e], hv.keys[2 * e + 1], a.seed) >> 32) & hv.imask;
        while (atomicCAS(&hv.index[i], kNoHeavy, e) != kNoHeavy) i = (i + 1) & hv.imask;
    }
    __syncthreads();
    return hv;
}

// Count the occurrence locally if its key is a heavy key (h = its table hash).
__device__ __forceinline__ bool heavy_count(const HeavyLds &hv, uint64_t h, const Occ &o) {
    uint32_t i = (uint32_t)(h >> 32) & hv.imask;
    while (true) {
        const uint32_t e = hv.index[i];
        if (e == kNoHeavy) return false;
        if (hv.keys[2 * e] == o.hi && hv.keys[2 * e + 1] == o.lo) {
            atomicAdd(&hv.cnt[9 * e + (o.left < 4 ? 1 + o.left : 0)], 1u);
            if (o.right < 4) atomicAdd(&hv.cnt[9 * e + 5 + o.right], 1u);
            return true;
        }
        i = (i + 1) & hv.imask;
    }
}

// Add the workgroup's heavy-key counts to the table: find (or insert) each
// key's slot once and add every non-zero counter to its wide counters.
// Called by every thread of the workgroup (contains a barrier).
template <int KW, bool CHECKED>
__device__ __forceinline__ void heavy_flush(const PassArgs &a, const HeavyLds &hv) {
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < hv.n; e += kBlock) {
        const uint32_t *c = hv.cnt + 9 * e;
        uint32_t any = 0;
        for (int q = 0; q < 9; ++q) any |= c[q];
        if (!any) continue;
        const uint64_t hi = hv.keys[2 * e], lo = hv.keys[2 * e + 1];
        const uint64_t h = key_hash(hi, lo, a.seed);
        uint64_t A, B;
        slot_words<KW>(hi, lo, A, B);
        const Probe pr = table_find<KW>(a.slots, a.cmask, h, A, B, a.max_probe, true);
        if (pr.slot < 0) {
            atomicOr(a.status, HM_ST_TABLE_FULL);
            continue;
        }
        if (pr.inserted && a.present) {
            uint64_t pw, pm;
            present_bits(h, a.present_mask, a.present_hash, pw, pm);
            __hip_atomic_fetch_or(a.present + pw, pm, RLX, AGT);
        }
        Slot *s = a.slots + pr.slot;
        for (int q = 0; q < 9; ++q) {
            if (!c[q]) continue;
            uint32_t *dst = q == 0 ? &s->nl : (q < 5 ? &s->tl[q - 1] : &s->tr[q - 5]);
            const uint32_t old = __hip_atomic_fetch_add(dst, c[q], RLX, AGT);
            if (CHECKED && old + c[q] < old) atomicOr(a.status, HM_ST_OVERFLOW);
        }
    }
}

// Per-occurrence body of pass 1.  `act` lanes carry an occurrence; every lane
// of the wave must call it (list appends are aggregated per wave).  With
// HEAVY, occurrences of the table's heavy keys are counted in `hv` instead.
// True when the filter lives in the table and a classification has since
// overwritten its words: pass 1 must then take every absent k-mer as seen (its
// earlier occurrences may have set bits that are gone).  Read once per launch.
__device__ __forceinline__ bool classified_in_table(const PassArgs &a) {
    if (a.bloom || a.bypass) return false;
    return (__builtin_amdgcn_readfirstlane(__hip_atomic_load(a.status, RLX, AGT)) & HM_ST_CLASSIFIED) != 0;
}

template <int KW, bool CHECKED, uint32_t CHUNK = kListChunk, bool HEAVY = false>
__device__ __forceinline__ void pass1_occ(const PassArgs &a, bool act, const Occ &o, ListCursor &cur, Stats &st,
                                          const HeavyLds *hv = nullptr, bool seen_all = false) {
    // The table is probed first: an occurrence whose k-mer is already there is
    // counted without touching the Bloom filter.  Only absent k-mers test and
    // set their Bloom bits; a k-mer the filter has seen is inserted and this
    // occurrence counted, an unseen one goes to the first-occurrence list.
    // The filter word is a word of the separate filter, or the home slot's
    // classification word, on the line the probe has just read.
    bool deferred = false;
    const uint64_t h = act ? key_hash(o.hi, o.lo, a.seed) : 0;
    if (HEAVY && act && heavy_count(*hv, h, o)) {
        st.v[HM_STAT_OCC] += 1;
        st.v[HM_STAT_HEAVY] += 1;
        act = false;
    }
    if (act) {
        uint64_t A, B;
        slot_words<KW>(o.hi, o.lo, A, B);
        Probe pr = table_find<KW>(a.slots, a.cmask, h, A, B, a.max_probe, a.bypass != 0);
        st.v[HM_STAT_OCC] += 1;
        st.v[HM_STAT_HIT] += pr.slot >= 0 ? 1u : 0u;
        if (pr.slot == -1) {
            st.v[HM_STAT_BLOOM] += 1;
            const uint64_t g = fmix64(h + 0x9E3779B97F4A7C15ull);
            bool seen;
            if (a.bloom) {
                uint64_t mask = 0;
                for (uint32_t j = 0; j < a.n_hash; ++j) mask |= 1ull << ((g >> (6 * j)) & 63);
                uint64_t *w = a.bloom + ((h >> 24) & a.bloom_mask);
                const uint64_t old = __hip_atomic_fetch_or(w, mask, RLX, AGT);
                seen = (old & mask) == mask;
            } else if (seen_all) {
                seen = true;
            } else {  // the home slot's classification word, on the line the probe just read
                uint32_t mask = 0;
                for (uint32_t j = 0; j < a.n_hash; ++j) mask |= 1u << ((g >> (5 * j)) & 31);
                uint32_t *w = &a.slots[h & a.cmask].cls;
                // Filter bits are only ever set while counting, so bits a plain (possibly stale) load
                // shows are set for good: a k-mer whose bits all show needs no atomic to know it was
                // seen.  Otherwise the atomic OR sets them and decides.
                seen = (*w & mask) == mask;
                if (!seen) seen = (__hip_atomic_fetch_or(w, mask, RLX, AGT) & mask) == mask;
            }
            if (seen) pr = table_find<KW>(a.slots, a.cmask, h, A, B, a.max_probe, true, pr.used);
            else deferred = true;
        }
        st.v[HM_STAT_DEFER] += deferred ? 1u : 0u;
        st.v[HM_STAT_PROBES] += pr.used + 1;
        st.v[HM_STAT_LINES] += pr.used / 2 + 1;  // steps 0-1 share the home line, then two per line
        if (pr.inserted && a.present) {
            uint64_t pw, pm;
            present_bits(h, a.present_mask, a.present_hash, pw, pm);
            __hip_atomic_fetch_or(a.present + pw, pm, RLX, AGT);
        }
        if (pr.slot >= 0) {
            const uint32_t c = count_occurrence<CHECKED>(a.slots + pr.slot, o.left, o.right, a.status, pr.narrow);
            st.v[HM_STAT_CAS] += c & 15;
            st.v[HM_STAT_WIDE] += c >= 16 ? 1u : 0u;
        } else if (pr.slot == -2) {
            atomicOr(a.status, HM_ST_TABLE_FULL);
        }
    }
    if (!a.bypass) {
        const bool need = deferred;
        const uint64_t m = __ballot(need);
        if (m) {
            const uint32_t n = (uint32_t)__popcll(m);
            const uint32_t pos = cur.used + lanes_below(m);
            uint64_t fresh = 0;
            if (cur.used + n > CHUNK) {  // wave-uniform: take a new chunk
                const int leader = __ffsll((long long)m) - 1;
                if ((int)lane_id() == leader) fresh = atomicAdd(a.lcount, (unsigned long long)CHUNK);
                fresh = __shfl(fresh, leader);
            }
            if (need) {
                const uint64_t idx = pos < CHUNK ? cur.base + pos : fresh + (pos - CHUNK);
                if (idx < a.lcap) {
                    a.lkeys[2 * idx] = o.hi;
                    a.lkeys[2 * idx + 1] = o.lo;
                    a.lext[idx] = (uint8_t)(o.left | (o.right << 4));
                } else {
                    atomicOr(a.status, HM_ST_LIST_FULL);
                }
            }
            cur.used += n;
            if (cur.used > CHUNK) {
                cur.base = fresh;
                cur.used -= CHUNK;
            }
        }
    }
}

// ------------------------------------------------------------------ window loops

// Visit every window of fixed-length reads, tile by tile: each tile's packed
// words are staged in the caller's LDS arrays (kTileB2Words / kTileMaskWords
// words).  op(act, occ, j) runs for every lane of the workgroup the same
// number of times per tile (act = the lane holds a valid, owned window;
// j = that window's base index in the read set).  With ABORT, a wave stops
// its tile once the table status says a pass failed.
template <bool ABORT, class Op>
__device__ __forceinline__ void fixed_windows(const PassArgs &a, int32_t reads_per_tile, int64_t n_tiles,
                                              uint64_t *s_b2, uint64_t *s_nm, uint64_t *s_hq, Op &&op) {
    const int L = a.read_len;
    const int k = a.k;
    const int W = L - k + 1;  // windows per read (> 0, checked by the host)
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t base0 = r0 * L, base1 = r1 * L;
        const int64_t org = base0 & ~(int64_t)63;              // origin: multiple of 64 bases
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
            if (ABORT && aborted(a.status)) break;
            const int f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            int64_t j = 0;
            if (f < total) {
                const int r = f / W;
                const int pos = f - r * W;
                const int64_t rb = (r0 + r) * L - org;
                act = extract(w, rb + pos, rb, rb + L, k, a.forward_only, a.n_owners, a.owner, o);
                j = (r0 + r) * L + pos;
            }
            op(act, o, j);
        }
    }
}

// Fixed-length reads with an owner filter.  Most windows belong to other
// owners, so counting each owned occurrence where it is found would keep one
// or two lanes of a wave busy with the table while the others wait.  Instead
// the owned occurrences are queued in LDS (one LDS atomic per wave per round)
// and handed to op a workgroup at a time, every lane holding one (act = false
// only in the last, partial round).  A full table is noticed per tile, for the
// whole workgroup, since the rounds meet at workgroup barriers.
constexpr unsigned kQueue = 512;  // a round adds at most kBlock: drained once more than kQueue - kBlock wait

struct OccQueue {
    uint4 *key;    // kQueue entries: (lo, hi) words of the canonical key
    uint8_t *ext;  // left | right << 4
    unsigned *n;
    int *stop;
};

template <bool ABORT, class Op>
__device__ __forceinline__ void fixed_windows_queued(const PassArgs &a, int32_t reads_per_tile, int64_t n_tiles,
                                                     uint64_t *s_b2, uint64_t *s_nm, uint64_t *s_hq,
                                                     const OccQueue &q, Op &&op) {
    const int L = a.read_len;
    const int k = a.k;
    const int W = L - k + 1;  // windows per read (> 0, checked by the host)
    const uint32_t lane = lane_id();
    auto drain = [&](unsigned n) {  // every thread calls it with the same n
        for (unsigned q0 = 0; q0 < n; q0 += kBlock) {
            const unsigned i = q0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            const bool act = i < n;
            if (act) {
                const uint4 kk = q.key[i];
                o.lo = ((uint64_t)kk.y << 32) | kk.x;
                o.hi = ((uint64_t)kk.w << 32) | kk.z;
                const uint8_t e = q.ext[i];
                o.left = e & 15;
                o.right = e >> 4;
            }
            op(act, o, (int64_t)0);
        }
    };
    if (threadIdx.x == 0) *q.n = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t base0 = r0 * L, base1 = r1 * L;
        const int64_t org = base0 & ~(int64_t)63;
        const int64_t mw0 = org >> 6;
        const int nmw = (int)(((base1 + 63) >> 6) - mw0) + 2;
        __syncthreads();  // previous tile's readers are done
        if (threadIdx.x == 0) *q.stop = ABORT && (__hip_atomic_load(a.status, RLX, AGT) & kAbortBits) != 0;
        for (int i = threadIdx.x; i < nmw; i += kBlock) {
            s_nm[i] = a.nm[mw0 + i];
            s_hq[i] = a.hq[mw0 + i];
        }
        for (int i = threadIdx.x; i < 2 * nmw; i += kBlock) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        if (*q.stop) break;  // workgroup-uniform
        const Words w{s_b2, s_nm, s_hq};
        const int total = (int)(r1 - r0) * W;
        for (int f0 = 0; f0 < total; f0 += kBlock) {  // workgroup-uniform trip count
            const int f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            if (f < total) {
                const int r = f / W;
                const int pos = f - r * W;
                const int64_t rb = (r0 + r) * L - org;
                act = extract(w, rb + pos, rb, rb + L, k, a.forward_only, a.n_owners, a.owner, o);
            }
            const uint64_t m = __ballot(act);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                unsigned base = 0;
                if ((int)lane == leader) base = atomicAdd(q.n, (unsigned)__popcll(m));
                base = __shfl(base, leader);
                if (act) {
                    const unsigned i = base + (unsigned)__popcll(m & ((1ull << lane) - 1));
                    q.key[i] = make_uint4((uint32_t)o.lo, (uint32_t)(o.lo >> 32), (uint32_t)o.hi,
                                          (uint32_t)(o.hi >> 32));
                    q.ext[i] = (uint8_t)(o.left | (o.right << 4));
                }
            }
            __syncthreads();  // the round's appends are done
            const unsigned n = *q.n;
            __syncthreads();  // every thread has read n before the count changes again
            if (n > kQueue - kBlock) {  // workgroup-uniform
                drain(n);
                __syncthreads();  // the entries are read before the next round overwrites them
                if (threadIdx.x == 0) *q.n = 0;
                __syncthreads();  // the cleared count is seen before the next round's appends
            }
        }
    }
    __syncthreads();
    const unsigned n = *q.n;
    drain(n);  // the rest (also after a stop: its occurrences were found before the table filled)
}

// ------------------------------------------------------------------ owned-occurrence stream writer

// A wave's stream space comes in chunks of kOccChunk entries, one atomic add
// each.  A write of n <= 64 entries (lane l the l-th) fills the current chunk
// and, when it runs out, continues in a fresh one, so entries are contiguous
// and the only holes are the tail of a wave's last chunk of a launch.
constexpr uint32_t kOccChunk = 1024;

struct OccOut {
    uint64_t *keys;  // 2 words per entry (hi, lo); 16-byte aligned
    uint8_t *ext;    // left | right << 4; kHole marks an unused entry
    uint64_t cap;
    unsigned long long *count;
};

struct OccCursor {  // wave-uniform
    uint64_t base;  // current chunk's first entry
    uint32_t used;  // entries of the chunk written (kOccChunk: no chunk yet)
};

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Write n (<= 64, wave-uniform) entries: lane l < n holds entry l (key words
// (hi lo32, hi hi32, lo lo32, lo hi32) and its extension byte).  Called by
// every lane of the wave.
__device__ __forceinline__ void occ_emit(const OccOut &out, OccCursor &cur, uint32_t n, uint4 key, uint8_t e) {
    const uint32_t l = lane_id();
    const uint32_t rem = kOccChunk - cur.used;
    uint64_t fresh = 0;
    if (n > rem) {
        unsigned long long b = 0;
        if (l == 0) b = atomicAdd(out.count, (unsigned long long)kOccChunk);
        fresh = __shfl(b, 0);
    }
    if (l < n) {
        const uint64_t idx = l < rem ? cur.base + cur.used + l : fresh + (l - rem);
        if (idx < out.cap) {
            *reinterpret_cast<uint4 *>(out.keys + 2 * idx) = key;
            out.ext[idx] = e;
        }
    }
    if (n > rem) {
        cur.base = fresh;
        cur.used = n - rem;
    } else {
        cur.used += n;
    }
}

// End of a wave's work: mark the rest of its chunk as holes.
__device__ __forceinline__ void occ_close(const OccOut &out, const OccCursor &cur) {
    if (cur.used >= kOccChunk) return;
    for (uint32_t i = cur.used + lane_id(); i < kOccChunk; i += 64) {
        const uint64_t idx = cur.base + i;
        if (idx < out.cap) out.ext[idx] = kHole;
    }
}

// A wave's staging ring in LDS (kRing entries): occurrences are appended by
// the lanes that hold one, and written 64 at a time with every lane busy.
constexpr uint32_t kRing = 128;  // a push adds <= 64 to fewer than 64 staged

struct OccRing {
    uint4 *key;
    uint32_t *aux;  // the ext byte, or what the caller needs to finish the entry
    uint32_t head, tail;  // wave-uniform: staged entries are [head, tail) mod kRing
};

// Stage the (key, aux) of every `act` lane (called by every lane of the wave).
__device__ __forceinline__ void ring_push(OccRing &g, bool act, uint64_t hi, uint64_t lo, uint32_t aux) {
    const uint64_t m = __ballot(act);
    if (act) {
        const uint32_t r = (g.tail + lanes_below(m)) & (kRing - 1);
        g.key[r] = make_uint4((uint32_t)hi, (uint32_t)(hi >> 32), (uint32_t)lo, (uint32_t)(lo >> 32));
        g.aux[r] = aux;
    }
    g.tail += (uint32_t)__popcll(m);
}

// Take the n (<= 64) oldest staged entries, lane l the l-th: returns whether
// the lane holds one (then `key` and `aux` are set).
__device__ __forceinline__ bool ring_take(OccRing &g, uint32_t n, uint4 &key, uint32_t &aux) {
    lds_wave_sync();  // every lane's staged entries are visible
    const uint32_t l = lane_id();
    const bool mine = l < n;
    if (mine) {
        const uint32_t r = (g.head + l) & (kRing - 1);
        key = g.key[r];
        aux = g.aux[r];
    }
    g.head += n;
    lds_wave_sync();  // the slots are read before later pushes reuse them
    return mine;
}

// Visit every window of variable-length reads (read_off given): packed words// Visit every window of variable-length reads (read_off given): packed words
// are read from global memory; a per-tile prefix sum in LDS (the caller's
// s_off / s_pre, kVarReads + 1 entries each) maps flat window indices to
// reads.  op as for fixed_windows.
template <bool ABORT, class Op>
__device__ __forceinline__ void var_windows(const PassArgs &a, int64_t n_tiles, int64_t *s_off, int64_t *s_pre,
                                            Op &&op) {
    const int k = a.k;
    const Words w{a.b2, a.nm, a.hq};
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
            if (ABORT && aborted(a.status)) break;
            const int64_t f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            int64_t j = 0;
            if (f < total) {
                int lo = 0, hi = nr;  // last read r with s_pre[r] <= f
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= f) lo = mid;
                    else hi = mid;
                }
                const int64_t rb = s_off[lo], re = max(s_off[lo + 1], rb);
                j = rb + (f - s_pre[lo]);
                act = extract(w, j, rb, re, k, a.forward_only, a.n_owners, a.owner, o);
            }
            op(act, o, j);
        }
    }
}

// Pass-2 body for one first-occurrence entry: skip it when the presence filter
// shows its k-mer was never inserted, else look it up and count it if found.
template <int KW, bool CHECKED>
__device__ __forceinline__ void pass2_entry(const PassArgs &a, uint64_t hi, uint64_t lo, uint8_t e, Stats &st) {
    st.v[HM_STAT_P2_ENTRIES] += 1;
    const uint64_t h = key_hash(hi, lo, a.seed);
    if (a.present) {
        uint64_t pw, pm;
        present_bits(h, a.present_mask, a.present_hash, pw, pm);
        if ((a.present[pw] & pm) != pm) return;  // never inserted: not in the table
    }
    uint64_t A, B;
    slot_words<KW>(hi, lo, A, B);
    const Probe pr = table_find<KW>(a.slots, a.cmask, h, A, B, a.max_probe, false);
    st.v[HM_STAT_P2_FOUND] += pr.slot >= 0 ? 1u : 0u;
    if (pr.slot >= 0) count_occurrence<CHECKED>(a.slots + pr.slot, e & 15, e >> 4, a.status, pr.narrow);
    else if (pr.slot == -2) atomicOr(a.status, HM_ST_TABLE_FULL);
}

// Mark the unused tail of the wave's current chunk as holes.
template <uint32_t CHUNK = kListChunk>
__device__ __forceinline__ void list_close(const PassArgs &a, const ListCursor &cur) {
    if (a.bypass || cur.used >= CHUNK) return;
    for (uint32_t i = cur.used + lane_id(); i < CHUNK; i += 64) {
        const uint64_t idx = cur.base + i;
        if (idx < a.lcap) a.lext[idx] = kHole;
    }
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

__device__ __forceinline__ uint64_t record_hash(uint64_t hi, uint64_t lo, uint32_t cnt, const uint32_t tl[4],
                                                const uint32_t tr[4], uint32_t cl, uint32_t cr) {
    uint64_t x = fmix64(hi ^ 0x6A09E667F3BCC908ull);
    x = fmix64(x ^ lo);
    x = fmix64(x ^ cnt);
    for (int b = 0; b < 4; ++b) x = fmix64(x ^ (((uint64_t)tl[b] << 32) | tr[b]));
    return fmix64(x ^ (cl | (cr << 8)));
}

// 16 bases of ASCII + Phred -> 2-bit codes and the two masks.
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


constexpr int kExportPerLane = 8;  // slots per lane per wave iteration: 512 per wave
constexpr int kExportChunk = 64 * kExportPerLane;

// Export one chunk of 64 * PER consecutive slots [first, first + 64 * PER) ∩
// [0, cap) with one wave: the slots are tested PER per lane (coalesced), the
// taken ones ranked with a wave prefix sum and their offsets staged in
// `rank_of` (LDS, 64 * PER entries per wave); one atomic add reserves the
// wave's output range and
// lane r writes record base+r, so every record store is coalesced.  With
// HM_EXPORT_CLASSIFY the depth filter and classes come from the counters
// (out.min_depth, out.ext_min); otherwise from the table's classify word.
// PER: slots per lane (the chunk is 64 * PER slots; the default 512).
template <int KW, int PER = kExportPerLane>
__device__ __forceinline__ void export_chunk(const Slot *slots, uint64_t first, uint64_t cap, uint32_t flags,
                                             const hm_export_t &out, uint32_t *status, uint16_t *rank_of,
                                             uint64_t &dsum, uint64_t &dxor, uint4 *staged = nullptr) {
    static_assert(PER >= 1 && PER <= 32, "one take bit per slot of a lane");
    const uint32_t lane = lane_id();
    const bool inline_cls = (flags & HM_EXPORT_CLASSIFY) != 0;
    uint32_t take_bits = 0;
#pragma unroll 1
    for (int j = 0; j < PER; ++j) {
        const uint64_t i = first + (uint64_t)j * 64 + lane;
        if (i < cap) {
            const Slot *sl = slots + i;
            if (sl->a != 0) {
                bool kept;
                uint32_t cl, cr;
                if (inline_cls) {
                    uint32_t tl[4], tr[4];
                    const uint64_t cnt = slot_counts(sl, tl, tr);
                    if (cnt > 0xFFFFFFFFull) atomicOr(status, HM_ST_OVERFLOW);
                    kept = cnt >= out.min_depth;
                    cl = side_class(tl, out.ext_min);
                    cr = side_class(tr, out.ext_min);
                } else {
                    const uint32_t c = sl->cls;
                    kept = (c >> 16) & 1;
                    cl = c & 0xFF;
                    cr = (c >> 8) & 0xFF;
                    if ((c >> 17) & 1) atomicOr(status, HM_ST_OVERFLOW);
                }
                bool take = (flags & HM_EXPORT_ALL) ? true : kept;
                if (flags & HM_EXPORT_UU_ONLY) take = take && kept && cl < 4 && cr < 4;
                take_bits |= (take ? 1u : 0u) << j;
            }
        }
    }
    const uint32_t cnt = (uint32_t)__popc(take_bits);
    uint32_t incl = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d);
        if ((int)lane >= d) incl += y;
    }
    const uint32_t total = __shfl(incl, 63);
    if (total == 0) return;
    uint32_t r = incl - cnt;
    for (int j = 0; j < PER; ++j)
        if ((take_bits >> j) & 1) rank_of[r++] = (uint16_t)(j * 64 + lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_out), (unsigned long long)total);
    base = __shfl(base, 0);
    for (uint32_t q = lane; q < total; q += 64) {
        const Slot *sl = slots + first + rank_of[q];
        uint64_t hi = 0, lo;
        if (KW == 1) {
            lo = sl->a & kLow63;
        } else {
            const uint64_t A = sl->a & kLow63, B = sl->b & kLow63;
            lo = B | (A << 63);
            hi = A >> 1;
        }
        uint32_t tl[4], tr[4];
        const uint32_t count = (uint32_t)slot_counts(sl, tl, tr);
        uint32_t cl, cr;
        if (inline_cls) {
            cl = side_class(tl, out.ext_min);
            cr = side_class(tr, out.ext_min);
        } else {
            const uint32_t c = sl->cls;
            cl = c & 0xFF;
            cr = (c >> 8) & 0xFF;
        }
        const uint64_t idx = base + q;
        if (idx < out.capacity) {
            out.key_hi[idx] = hi;
            out.key_lo[idx] = lo;
            if (staged) {  // a key-ordered export: the sort gathers these into place
                staged[4 * idx] = make_uint4(tl[0], tl[1], tl[2], tl[3]);
                staged[4 * idx + 1] = make_uint4(tr[0], tr[1], tr[2], tr[3]);
                staged[4 * idx + 2] = make_uint4(count, cl | (cr << 8), 0u, 0u);
            } else {
                out.count[idx] = count;
                *reinterpret_cast<uint4 *>(out.tl + 4 * idx) = make_uint4(tl[0], tl[1], tl[2], tl[3]);
                *reinterpret_cast<uint4 *>(out.tr + 4 * idx) = make_uint4(tr[0], tr[1], tr[2], tr[3]);
                out.cls_l[idx] = (uint8_t)cl;
                out.cls_r[idx] = (uint8_t)cr;
            }
        } else {
            atomicOr(status, HM_ST_OUTPUT_FULL);
        }
        if (out.digest) {
            const uint64_t x = record_hash(hi, lo, count, tl, tr, cl, cr);
            dsum += x;
            dxor ^= x;
        }
    }
    __builtin_amdgcn_wave_barrier();  // rank_of is rewritten by the next chunk
}

// Add a wave's digest terms to the export digest.
__device__ __forceinline__ void digest_flush(const hm_export_t &out, uint64_t dsum, uint64_t dxor) {
    if (!out.digest) return;
    for (int off = 32; off > 0; off >>= 1) {
        dsum += __shfl_xor(dsum, off);
        dxor ^= __shfl_xor(dxor, off);
    }
    if (lane_id() == 0 && (dsum | dxor)) {
        atomicAdd(reinterpret_cast<unsigned long long *>(out.digest), (unsigned long long)dsum);
        atomicXor(reinterpret_cast<unsigned long long *>(out.digest + 1), (unsigned long long)dxor);
    }
}

// ------------------------------------------------------------------ host helpers (defined in hm_kmer.hip)

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int device_cus();
inline bool pow2(uint64_t x) { return x && !(x & (x - 1)); }
uint64_t grid_for(uint64_t items, int per_cu = 8);
// argument checks shared by the entry points (defined in hm_kmer.hip)
int check_reads(const hm_reads_t *r, int k);
int check_table(const hm_table_t *t);
int check_occ(const hm_occ_t *o);
// key-order sort of an export (defined in hm_sort.hip); key_bits = 2k.  The
// export writes each record's counters and classes into sort_staging(out)
// (one 64-byte line per record), from where the sort gathers them.
uint64_t sort_work_bytes(uint64_t capacity);
uint4 *sort_staging(const hm_export_t &out);
int sort_export(const hm_export_t &out, int key_bits, hipStream_t s);

#define HM_LAUNCH_CHECK(what)                                \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) return hm::hip_fail(e_, what); \
    } while (0)

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, uint64_t n, T v) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) p[i] = v;
}

template <typename T>
int fill(T *p, uint64_t n, T v, hipStream_t s) {
    if (n == 0) return HM_OK;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)grid_for(n, 16)), dim3(kBlock), 0, s, p, n, v);
    HM_LAUNCH_CHECK("fill");
    return HM_OK;
}

}  // namespace hm
