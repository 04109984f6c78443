// hm_bins.hip -- binned counting: the owner-computes decomposition of section
// "Parallel k-mer analysis" inside one GPU.
//
// The paper assigns every k-mer to one processor by a hash of the k-mer, ships
// each occurrence to its owner, and each owner filters its share with a Bloom
// filter and counts it in a hash table of its own.  Here the owners are bins
// small enough for one workgroup's local memory (LDS): the occurrences are
// partitioned by a hash of their canonical key into 2^(group_bits + bin_bits)
// bins (two counting-sort passes over 16-byte records, exact offsets from
// histograms, so no record moves through an atomic queue), and then one
// workgroup at a time takes a bin and runs the same two-pass method on it in
// LDS: an occurrence whose k-mer is already in the bin's table is counted; an
// absent k-mer tests and sets its bits in the bin's Bloom filter, a k-mer the
// filter has seen is inserted and counted, an unseen one is deferred and
// counted after the bin's last occurrence if its k-mer is in the table by
// then.  Depth filter, classification and export follow straight from LDS.
// The table, filter and counters never touch HBM, so the path streams records
// instead of making one random device-scope atomic per occurrence.
//
// A bin whose table would pass three quarters full, or whose deferred
// occurrences pass the LDS list, is not counted here: its records are copied
// to an occurrence stream (hm_occ_t) for the global-table path
// (hm_bloom_insert_occ, hm_kmer_count, hm_export_table), whose export
// hm_export_merge appends to this one.  Either way every occurrence is counted
// exactly once, whatever the Bloom false positives.
#include <mutex>
#include <unordered_map>

#include "hm_bins.h"
#include "hm_roll.h"

namespace hm {
namespace {

#ifndef HM_BIN_GRID1
#define HM_BIN_GRID1 1024
#endif
constexpr int kGrid1 = HM_BIN_GRID1;  // most workgroups of the two passes over the reads
constexpr int kSlices = 8;         // workgroups per group in the second partition level
constexpr int kMaxGroupBits = 10;  // LDS of the first-level scatter's combiner
constexpr int kMaxBinBits = 11;    // LDS of the second-level scatter's combiner
#ifndef HM_BIN_BLK1
#define HM_BIN_BLK1 8
#endif
#ifndef HM_BIN_BLK2
#define HM_BIN_BLK2 4
#endif
constexpr int kBlk1 = HM_BIN_BLK1;  // records per written block, first level
constexpr int kBlk2 = HM_BIN_BLK2;  // records per written block, second level
constexpr int kT2 = 1024;           // threads of a second-level workgroup
#ifndef HM_BIN_FLUSH1
#define HM_BIN_FLUSH1 1024
#endif
#ifndef HM_BIN_T1
#define HM_BIN_T1 512
#endif
constexpr int kT1 = HM_BIN_T1;               // threads of a first-level scatter workgroup
constexpr int kFlush1 = HM_BIN_FLUSH1 / kT1;  // first level: rounds between flushes (HM_BIN_FLUSH1 windows)
static_assert(kFlush1 >= 1, "flush at most once a round");
constexpr int kBinSlots = 512;     // LDS table of one bin
#ifndef HM_BIN_BLOOM_WORDS
#define HM_BIN_BLOOM_WORDS 512
#endif
#ifndef HM_BIN_DEFER_CAP
#define HM_BIN_DEFER_CAP 2048
#endif
constexpr int kBloomWords = HM_BIN_BLOOM_WORDS;  // 32-bit filter words: 16384 bits per bin
constexpr int kDeferCap = HM_BIN_DEFER_CAP;  // deferred occurrences of one bin
constexpr int kPer = 4;            // records per thread per round (second-level histogram)
constexpr int kChunk = kPer * kBlock;
#ifndef HM_BIN_COUNT_PER
#define HM_BIN_COUNT_PER 2
#endif
constexpr int kCPer = HM_BIN_COUNT_PER;  // records per thread per round of the counting pass
constexpr int kCChunk = kCPer * kBlock;
constexpr uint32_t kMaxKeys = kBinSlots * 3 / 4;
constexpr int kExtShift = 58;
constexpr int kMaxBinK = 61;       // 2k + 6 extension bits fit in 128
#ifndef HM_BIN_COUNT_PER_CU
#define HM_BIN_COUNT_PER_CU 4
#endif
constexpr int kCountBlocksPerCu = HM_BIN_COUNT_PER_CU;
static_assert(kBinSlots == 2 * kBlock, "the export takes two slots a thread");


// record: word 0 = key_lo, word 1 = key_hi | ext << 58, ext = left | right << 3 (0..3 base, 4 none)
__device__ __forceinline__ uint4 rec_pack(const Occ &o) {
    const uint64_t w1 = o.hi | ((uint64_t)(o.left | (o.right << 3)) << kExtShift);
    return make_uint4((uint32_t)o.lo, (uint32_t)(o.lo >> 32), (uint32_t)w1, (uint32_t)(w1 >> 32));
}

struct Rec {
    uint64_t hi, lo;
    int left, right;
};

__device__ __forceinline__ Rec rec_unpack(uint4 r) {
    Rec x;
    x.lo = ((uint64_t)r.y << 32) | r.x;
    const uint64_t w1 = ((uint64_t)r.w << 32) | r.z;
    x.hi = w1 & ((1ull << kExtShift) - 1);
    const int e = (int)(w1 >> kExtShift);
    x.left = e & 7;
    x.right = e >> 3;
    return x;
}

// ------------------------------------------------------------------ partition

// A hole: padding that keeps every destination range a whole number of blocks (word 3 has the
// extension field 63, which no record has); readers skip it.
__device__ __forceinline__ bool is_hole(uint4 r) { return (r.w >> (kExtShift - 32)) == 63u; }
__device__ __forceinline__ uint4 hole_rec() { return make_uint4(0u, 0u, 0u, 0xFFFFFFFFu); }

// Write-combining of 16-byte records into F destinations, each a range of a global array that
// starts at a multiple of BLK records and is padded with holes to a multiple of BLK.  Each
// destination keeps a ring of BLK records in LDS; a round of put() calls is followed (after a
// barrier) by flush(), which writes every completed block with BLK consecutive stores, so HBM
// sees whole blocks instead of one partial line per record.  A record whose block is not the
// ring's current one (its destination took more than a block in one round) is stored at once.
template <int BLK>
struct Combiner {
    uint4 *ring;        // F * BLK
    uint32_t *fill;     // records placed, relative to the destination's start
    uint32_t *done;     // records written out in whole blocks (a multiple of BLK)
    uint8_t *bits;      // ring entries that hold a record
    uint16_t *ready;    // destinations whose block filled up this round
    uint32_t *n_ready;  // two counters: rounds alternate between them
    // LDS bytes for F destinations
    static constexpr size_t bytes(size_t F) {
        return F * (BLK * 16 + 8) + 2 * ((F + 1) & ~(size_t)1) + ((F + 3) & ~(size_t)3) + 8;
    }
    // carve the arrays from `lds` (16-byte aligned) for F destinations; returns the first free byte
    __device__ uint8_t *carve(void *lds, int F) {
        ring = reinterpret_cast<uint4 *>(lds);
        fill = reinterpret_cast<uint32_t *>(ring + (size_t)F * BLK);
        done = fill + F;
        ready = reinterpret_cast<uint16_t *>(done + F);
        bits = reinterpret_cast<uint8_t *>(ready + ((F + 1) & ~1));
        n_ready = reinterpret_cast<uint32_t *>(bits + ((F + 3) & ~3));
        return reinterpret_cast<uint8_t *>(n_ready + 2);
    }
    // round `par` (0 or 1, alternating)
    __device__ void put(uint32_t d, uint4 r, uint4 *at, uint32_t par) {  // at: the destination's first record
        const uint32_t p = atomicAdd(&fill[d], 1u);
        const uint32_t q = p - done[d];
        if (q < (uint32_t)BLK) {
            ring[d * BLK + q] = r;
            atomicOr(reinterpret_cast<uint32_t *>(bits + (d & ~3u)), 1u << (8 * (d & 3) + q));
            if (q == BLK - 1) ready[atomicAdd(&n_ready[par], 1u)] = (uint16_t)d;  // the block is complete
        } else {
            at[p] = r;
        }
    }
    // after a barrier: write out the completed blocks of the round's ready destinations and clear
    // the other round's counter (then a barrier before the next round)
    template <class At>
    __device__ void flush_ready(uint32_t tid, uint32_t nthreads, At at, uint32_t par) {
        if (tid == 0) n_ready[par ^ 1] = 0;
        const uint32_t n = n_ready[par];
        for (uint32_t i = tid; i < n; i += nthreads) {
            const uint32_t d = ready[i];
            uint4 *o = at(d);
            const uint32_t f = fill[d];
            uint32_t dn = done[d], b = bits[d];
            const uint4 *src = ring + d * BLK;
            while (f - dn >= (uint32_t)BLK) {
                if (b == (1u << BLK) - 1) {
#pragma unroll
                    for (int q = 0; q < BLK; ++q) o[dn + q] = src[q];
                } else {
                    for (int q = 0; q < BLK; ++q)
                        if ((b >> q) & 1) o[dn + q] = src[q];
                }
                b = 0;
                dn += BLK;
            }
            done[d] = dn;
            bits[d] = (uint8_t)b;
        }
    }
    __device__ void flush_tail(uint32_t d, uint4 *at) {  // the last block, padded with holes
        const uint32_t f = fill[d], dn = done[d], b = bits[d];
        if (f == dn) return;
        const uint4 *src = ring + d * BLK;
#pragma unroll
        for (int q = 0; q < BLK; ++q) {
            const uint32_t p = dn + q;
            if (p >= f) at[p] = hole_rec();
            else if ((b >> q) & 1) at[p] = src[q];
        }
    }
};

// Every window of the fixed-length reads of this workgroup's tiles (tile = blockIdx.x, then
// every gridDim.x-th: they depend only on the grid), a run of kCardRun windows per lane, handed
// to op(act, occurrence) in rounds the whole workgroup takes together: round i gives every lane
// its run's window i, act false where the window holds an invalid base, is past the read's last
// window or has another owner.  The key is the canonical one, with the extensions pass 1 takes.
template <int KW, int NT, class Op>
__device__ __forceinline__ void fixed_runs(const PassArgs &a, int32_t reads_per_tile, int64_t n_tiles, uint64_t *s_b2,
                                           uint64_t *s_nm, uint64_t *s_hq, Op &&op) {
    const int L = a.read_len, k = a.k;
    const int W = L - k + 1;  // > 0, checked by the host
    const int runs = (W + kCardRun - 1) / kCardRun;
    const typename Roll<KW>::Shape sh = Roll<KW>::shape(k);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t org = (r0 * L) & ~(int64_t)63;
        const int64_t mw0 = org >> 6;
        const int nmw = (int)((((r1 * L) + 63) >> 6) - mw0) + 2;  // incl. 2 guard words
        __syncthreads();  // the previous tile's readers are done
        for (int i = threadIdx.x; i < nmw; i += NT) {
            s_nm[i] = a.nm[mw0 + i];
            s_hq[i] = a.hq[mw0 + i];
        }
        for (int i = threadIdx.x; i < 2 * nmw; i += NT) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        const Words w{s_b2, s_nm, s_hq};
        const int total = (int)(r1 - r0) * runs;
        for (int g0 = 0; g0 < total; g0 += NT) {  // workgroup-uniform
            const int g = g0 + (int)threadIdx.x;
            int cnt = 0;
            int64_t j0 = 0, rb = 0;
            uint32_t vm = 0;
            RunBits bits;
            RunExt ext;
            Roll<KW> x;
            if (g < total) {
                const int r = g / runs;
                const int p0 = (g - r * runs) * kCardRun;
                cnt = min(kCardRun, W - p0);
                rb = (r0 + r) * L - org;
                j0 = rb + p0;
                bits.load(w, j0, k);
                vm = bits.valid_mask(k, cnt);
                ext.load(w, j0, k);
                const U128 f = w.window(j0, k);
                x.set(f, revcomp(f, k));
            }
#pragma unroll 1
            for (int i = 0; i < kCardRun; ++i) {  // round i
                Occ o{0, 0, 4, 4};
                bool act = false;
                if (i < cnt) {
                    if (i > 0) x.step((uint32_t)bits.base(i), sh);
                    if ((vm >> i) & 1u) {
                        const bool fwd = a.forward_only || x.forward();
                        int left, right;
                        ext.fwd_ext(bits, i, j0, rb, rb + L, k, left, right);
                        o.hi = fwd ? x.fhi() : x.rhi();
                        o.lo = fwd ? x.flo() : x.rlo();
                        o.left = fwd ? left : (right < 4 ? 3 - right : 4);
                        o.right = fwd ? right : (left < 4 ? 3 - left : 4);
                        act = a.n_owners <= 1 || owner_of(o.hi, o.lo, a.n_owners) == a.owner;
                    }
                }
                op(act, o);
            }
        }
    }
}

// Level-1 histogram: counts of each group's windows in this workgroup's tiles (the same tiles
// and windows as the scatter pass with the same grid), into hist1[blockIdx.x * groups + group].
template <int KW>
__global__ __launch_bounds__(kBlock) void k_hist1(PassArgs a, int32_t rpt, int64_t n_tiles, uint32_t *hist1,
                                                  int total_bits, int bin_bits) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    extern __shared__ uint32_t s_h[];
    const int ng = 1 << (total_bits - bin_bits);
    for (int i = threadIdx.x; i < ng; i += kBlock) s_h[i] = 0;
    fixed_runs<KW, kBlock>(a, rpt, n_tiles, s_b2, s_nm, s_hq, [&](bool act, const Occ &o) {
        if (act) atomicAdd(&s_h[bin_of(o.hi, o.lo, total_bits) >> bin_bits], 1u);
    });
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += kBlock) hist1[(size_t)blockIdx.x * ng + i] = s_h[i];
}

// Exclusive prefix sum, in place, of each row of x (rows x cols, one workgroup per row) over
// the counts rounded up to a multiple of `pad`; the row total to tot[row].  Every row total is
// below 2^32 (checked by the host).
__global__ __launch_bounds__(kBlock) void k_scan_rows(uint32_t *x, int cols, uint32_t pad, uint64_t *tot) {
    __shared__ uint32_t s_part[kBlock];
    uint32_t *row = x + (size_t)blockIdx.x * cols;
    const int per = (cols + kBlock - 1) / kBlock;
    const int b = min((int)threadIdx.x * per, cols), e = min(b + per, cols);
    uint32_t sum = 0;
    for (int i = b; i < e; ++i) sum += (row[i] + pad - 1) / pad * pad;
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {  // inclusive scan of the thread sums
        const uint32_t y = (int)threadIdx.x >= d ? s_part[threadIdx.x - d] : 0u;
        __syncthreads();
        s_part[threadIdx.x] += y;
        __syncthreads();
    }
    uint32_t run = s_part[threadIdx.x] - sum;
    for (int i = b; i < e; ++i) {
        const uint32_t v = (row[i] + pad - 1) / pad * pad;
        row[i] = run;
        run += v;
    }
    if (tot && threadIdx.x == kBlock - 1) tot[blockIdx.x] = s_part[kBlock - 1];
}

// start[i] = sum of tot[0..i), i = 0..n (one workgroup; n: groups or first-level workgroups)
__global__ __launch_bounds__(kBlock) void k_scan_totals(const uint64_t *tot, int n, uint64_t *start) {
    __shared__ uint64_t s_part[kBlock];
    const int per = (n + kBlock - 1) / kBlock;
    const int b = min((int)threadIdx.x * per, n), e = min(b + per, n);
    uint64_t sum = 0;
    for (int i = b; i < e; ++i) sum += tot[i];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        const uint64_t y = (int)threadIdx.x >= d ? s_part[threadIdx.x - d] : 0ull;
        __syncthreads();
        s_part[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = s_part[threadIdx.x] - sum;
    for (int i = b; i < e; ++i) {
        start[i] = run;
        run += tot[i];
    }
    if (threadIdx.x == kBlock - 1) start[n] = s_part[kBlock - 1];
}

// Level-1 scatter: the same windows as k_hist1, through a combiner per group, into this
// workgroup's own region of tmp (from wstart[blockIdx.x]), where each group has a piece at the
// offset rel1[blockIdx.x * groups + group].  One region a workgroup keeps the pages its stores
// touch few: with a range per group spread over the whole buffer, nearly every store missed the
// address translation cache.
template <int KW>
__global__ __launch_bounds__(kT1) void k_scatter1(PassArgs a, int32_t rpt, int64_t n_tiles, const uint32_t *rel1,
                                                  const uint64_t *wstart, uint4 *tmp, int total_bits, int bin_bits) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    extern __shared__ uint4 s_dyn[];
    const int ng = 1 << (total_bits - bin_bits);
    Combiner<kBlk1> cb;
    // each group's piece (below 2^32 records, checked by the host), in LDS so that the put path
    // makes no global load
    uint32_t *s_at = reinterpret_cast<uint32_t *>(cb.carve(s_dyn, ng));
    const uint64_t region = wstart[blockIdx.x];
    for (int i = threadIdx.x; i < ng; i += kT1) {
        s_at[i] = (uint32_t)(region + rel1[(size_t)blockIdx.x * ng + i]);
        cb.fill[i] = cb.done[i] = 0;
        cb.bits[i] = 0;
    }
    if (threadIdx.x < 2) cb.n_ready[threadIdx.x] = 0;
    auto at = [&](uint32_t g) { return tmp + s_at[g]; };
    uint32_t par = 0, round = 0;
    fixed_runs<KW, kT1>(a, rpt, n_tiles, s_b2, s_nm, s_hq, [&](bool act, const Occ &o) {
        if (act) {
            const uint32_t g = bin_of(o.hi, o.lo, total_bits) >> bin_bits;
            cb.put(g, rec_pack(o), at(g), par);
        }
        if (++round == (uint32_t)kFlush1) {  // workgroup-uniform
            round = 0;
            __syncthreads();
            cb.flush_ready(threadIdx.x, kT1, at, par);
            __syncthreads();
            par ^= 1;
        }
    });
    __syncthreads();
    cb.flush_ready(threadIdx.x, kT1, at, par);  // blocks completed since the last flush
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += kT1) cb.flush_tail(g, at(g));
}

// The first level over an occurrence stream (hm_occ_t: the owned occurrences a cardinality pass
// wrote) instead of over the reads: workgroup w takes the entries [w * per, (w + 1) * per) of the
// n = min(count, capacity) reserved ones, per = ceil(n / gridDim.x), NT a round (the entries of
// four rounds loaded together), and hands each to op(act, record); holes (ext 0xFF) and positions
// past the chunk come with act false.  The histogram pass and the scatter pass use the same grid,
// so they see the same chunks.
template <int NT, class Op>
__device__ __forceinline__ void occ_rounds(const hm_occ_t &o, Op &&op) {
    constexpr int kAhead = 4;  // rounds whose entries are loaded together
    const uint64_t n = min(*o.count, o.capacity);
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = min(n, (uint64_t)blockIdx.x * per), e = min(n, b + per);
    const uint4 *keys = reinterpret_cast<const uint4 *>(o.keys);
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kAhead) {  // workgroup-uniform
        uint4 kk[kAhead];
        uint32_t x[kAhead];
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            const uint64_t i = i0 + (uint64_t)j * NT + threadIdx.x;
            x[j] = i < e ? o.ext[i] : kHole;
            kk[j] = i < e ? keys[i] : make_uint4(0, 0, 0, 0);  // key_hi, key_lo as four 32-bit words
        }
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            if (i0 + (uint64_t)j * NT >= e) break;  // workgroup-uniform: no round past the chunk
            const uint32_t ext = (x[j] & 15u) | ((x[j] >> 4) << 3);
            op(x[j] != kHole, make_uint4(kk[j].z, kk[j].w, kk[j].x, kk[j].y | (ext << (kExtShift - 32))));
        }
    }
}

__device__ __forceinline__ uint32_t rec_bin(uint4 r, int total_bits) {
    const uint64_t lo = ((uint64_t)r.y << 32) | r.x;
    const uint64_t hi = (((uint64_t)r.w << 32) | r.z) & ((1ull << kExtShift) - 1);
    return bin_of(hi, lo, total_bits);
}

// Level-1 histogram over a stream: hist1[blockIdx.x * groups + group].  The chunks are those of
// occ_rounds (they depend on the grid alone); a pure stream, so 1024 threads a workgroup and
// kHistPer entries a thread in flight.
constexpr int kHistT = 1024, kHistPer = 4;

__global__ __launch_bounds__(kHistT) void k_hist1_occ(hm_occ_t o, uint32_t *hist1, int total_bits, int bin_bits) {
    extern __shared__ uint32_t s_h[];
    const int ng = 1 << (total_bits - bin_bits);
    for (int i = threadIdx.x; i < ng; i += kHistT) s_h[i] = 0;
    __syncthreads();
    const uint64_t n = min(*o.count, o.capacity);
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = min(n, (uint64_t)blockIdx.x * per), e = min(n, b + per);
    const uint4 *keys = reinterpret_cast<const uint4 *>(o.keys);
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)kHistT * kHistPer) {
        uint4 kk[kHistPer];
        uint32_t x[kHistPer];
#pragma unroll
        for (int j = 0; j < kHistPer; ++j) {
            const uint64_t i = i0 + (uint64_t)j * kHistT + threadIdx.x;
            x[j] = i < e ? o.ext[i] : kHole;
            kk[j] = i < e ? keys[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < kHistPer; ++j) {
            if (x[j] == kHole) continue;
            const uint64_t hi = ((uint64_t)kk[j].y << 32) | kk[j].x, lo = ((uint64_t)kk[j].w << 32) | kk[j].z;
            atomicAdd(&s_h[bin_of(hi, lo, total_bits) >> bin_bits], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += kHistT) hist1[(size_t)blockIdx.x * ng + i] = s_h[i];
}

// Level-1 scatter over a stream: as k_scatter1, from the workgroup's chunk of entries.
__global__ __launch_bounds__(kT1) void k_scatter1_occ(hm_occ_t o, const uint32_t *rel1, const uint64_t *wstart,
                                                      uint4 *tmp, int total_bits, int bin_bits) {
    extern __shared__ uint4 s_dyn[];
    const int ng = 1 << (total_bits - bin_bits);
    Combiner<kBlk1> cb;
    uint32_t *s_at = reinterpret_cast<uint32_t *>(cb.carve(s_dyn, ng));
    const uint64_t region = wstart[blockIdx.x];
    for (int i = threadIdx.x; i < ng; i += kT1) {
        s_at[i] = (uint32_t)(region + rel1[(size_t)blockIdx.x * ng + i]);
        cb.fill[i] = cb.done[i] = 0;
        cb.bits[i] = 0;
    }
    if (threadIdx.x < 2) cb.n_ready[threadIdx.x] = 0;
    __syncthreads();
    auto at = [&](uint32_t g) { return tmp + s_at[g]; };
    uint32_t par = 0, round = 0;
    occ_rounds<kT1>(o, [&](bool act, uint4 r) {
        if (act) {
            const uint32_t g = rec_bin(r, total_bits) >> bin_bits;
            cb.put(g, r, at(g), par);
        }
        if (++round == (uint32_t)kFlush1) {  // workgroup-uniform
            round = 0;
            __syncthreads();
            cb.flush_ready(threadIdx.x, kT1, at, par);
            __syncthreads();
            par ^= 1;
        }
    });
    __syncthreads();
    cb.flush_ready(threadIdx.x, kT1, at, par);
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += kT1) cb.flush_tail(g, at(g));
}

// The second level's input: group g's records lie in pieces, one per first-level workgroup w,
// from wstart[w] + rel1[w * ng + g] to the next group's piece (the workgroup's region's end for
// the last group).  Second-level workgroup (g, slice) takes the pieces of first-level workgroups
// [slice * g1 / kSlices, (slice + 1) * g1 / kSlices) as one run of positions: vs[j] is where piece
// j starts in the run (vs[n] its length), ad[j] where it starts in tmp.  Returns the length.
constexpr int kMaxPieces = (kGrid1 + kSlices - 1) / kSlices;

__device__ uint32_t load_pieces(const uint32_t *rel1, const uint64_t *wstart, int ng, int g1, uint32_t g,
                                uint32_t sl, uint32_t *vs, uint32_t *ad, int &n) {
    const int w0 = (int)(sl * (uint32_t)g1 / kSlices), w1 = (int)((sl + 1) * (uint32_t)g1 / kSlices);
    n = w1 - w0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int w = w0 + j;
        const uint64_t b = wstart[w] + rel1[(size_t)w * ng + g];
        const uint64_t e = g + 1 < (uint32_t)ng ? wstart[w] + rel1[(size_t)w * ng + g + 1] : wstart[w + 1];
        ad[j] = (uint32_t)b;  // below 2^32 records (checked by the host)
        vs[j] = (uint32_t)(e - b);
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // at most kMaxPieces lengths
        uint32_t run = 0;
        for (int j = 0; j < n; ++j) {
            const uint32_t len = vs[j];
            vs[j] = run;
            run += len;
        }
        vs[n] = run;
    }
    __syncthreads();
    return vs[n];
}

// tmp index of position v (< the run's length) of the run of pieces, in the last piece starting at
// or before v (a non-empty one).  A thread asks for increasing positions, so its piece index p
// (start it at 0) only moves forward, past empty pieces too.
__device__ __forceinline__ uint32_t piece_at(const uint32_t *vs, const uint32_t *ad, int n, uint32_t v, int &p) {
    while (p + 1 < n && vs[p + 1] <= v) ++p;
    return ad[p] + (v - vs[p]);
}

// Level-2 histogram: workgroup (g, slice) counts the bins of its slice of group g's records.
__global__ __launch_bounds__(kBlock) void k_hist2(const uint4 *tmp, const uint32_t *rel1, const uint64_t *wstart,
                                                  int g1, uint32_t *hist2, int total_bits, int bin_bits) {
    extern __shared__ uint32_t s_h[];
    __shared__ uint32_t s_vs[kMaxPieces + 1], s_ad[kMaxPieces];
    const int ns = 1 << bin_bits, ng = 1 << (total_bits - bin_bits);
    const uint32_t g = blockIdx.x / kSlices, sl = blockIdx.x % kSlices;
    for (int i = threadIdx.x; i < ns; i += kBlock) s_h[i] = 0;
    int n;
    const uint32_t len = load_pieces(rel1, wstart, ng, g1, g, sl, s_vs, s_ad, n);  // starts with a barrier
    const uint32_t mask = (uint32_t)ns - 1;
    int pc = 0;  // this thread's piece
    for (uint32_t v0 = 0; v0 < len; v0 += kChunk) {
        uint4 r[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t v = v0 + j * kBlock + threadIdx.x;
            r[j] = v < len ? tmp[piece_at(s_vs, s_ad, n, v, pc)] : hole_rec();
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (is_hole(r[j])) continue;
            const Rec x = rec_unpack(r[j]);
            atomicAdd(&s_h[bin_of(x.hi, x.lo, total_bits) & mask], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns; i += kBlock) hist2[((size_t)g * ns + i) * kSlices + sl] = s_h[i];
}

// bin_start[g * ns + s] = group start (in recs) + offset of (s, slice 0) within the group; the
// last entry closes the final bin.
__global__ __launch_bounds__(kBlock) void k_bin_starts(const uint32_t *rel2, const uint64_t *gstart2,
                                                       uint64_t *bin_start, int total_bits, int bin_bits) {
    const uint64_t n_bins = 1ull << total_bits;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i <= n_bins; i += (uint64_t)gridDim.x * kBlock) {
        if (i == n_bins) bin_start[i] = gstart2[n_bins >> bin_bits];
        else bin_start[i] = gstart2[i >> bin_bits] + rel2[i * kSlices];
    }
}

// Level-2 scatter: workgroup (g, slice) rereads its slice and places each record in its bin's
// range at the slice's offset, through a combiner per bin.
__global__ __launch_bounds__(kT2) void k_scatter2(const uint4 *tmp, const uint32_t *rel1, const uint64_t *wstart, int g1,
                                                  const uint64_t *gstart2, const uint32_t *rel2, uint4 *recs,
                                                  int total_bits, int bin_bits) {
    extern __shared__ uint4 s_dyn[];
    __shared__ uint32_t s_vs[kMaxPieces + 1], s_ad[kMaxPieces];
    const int ns = 1 << bin_bits, ng = 1 << (total_bits - bin_bits);
    const uint32_t g = blockIdx.x / kSlices, sl = blockIdx.x % kSlices;
    Combiner<kBlk2> cb;
    uint32_t *s_rel = reinterpret_cast<uint32_t *>(cb.carve(s_dyn, ns));
    for (int i = threadIdx.x; i < ns; i += kT2) {
        s_rel[i] = rel2[((size_t)g * ns + i) * kSlices + sl];
        cb.fill[i] = cb.done[i] = 0;
        cb.bits[i] = 0;
    }
    if (threadIdx.x < 2) cb.n_ready[threadIdx.x] = 0;
    int n;
    const uint32_t len = load_pieces(rel1, wstart, ng, g1, g, sl, s_vs, s_ad, n);  // starts with a barrier
    uint32_t par = 0;
    uint4 *base = recs + gstart2[g];
    auto at = [&](uint32_t d) { return base + s_rel[d]; };
    const uint32_t mask = (uint32_t)ns - 1;
    int pc = 0;  // this thread's piece
    for (uint32_t v0 = 0; v0 < len; v0 += 2 * kT2) {
        uint4 r[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t v = v0 + j * kT2 + threadIdx.x;
            r[j] = v < len ? tmp[piece_at(s_vs, s_ad, n, v, pc)] : hole_rec();
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (is_hole(r[j])) continue;
            const Rec x = rec_unpack(r[j]);
            const uint32_t d = bin_of(x.hi, x.lo, total_bits) & mask;
            cb.put(d, r[j], at(d), par);
        }
        __syncthreads();
        cb.flush_ready(threadIdx.x, kT2, at, par);
        __syncthreads();
        par ^= 1;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ns; d += kT2) cb.flush_tail(d, at(d));
}

// ------------------------------------------------------------------ counting in LDS

constexpr int kStage = 2048;               // records a workgroup stages before it takes an output range
#ifndef HM_BIN_COUNT_GRID
#define HM_BIN_COUNT_GRID 1024
#endif
constexpr int kCountGrid = HM_BIN_COUNT_GRID;  // most workgroups of hm_count_bins (one staging area each)
constexpr uint64_t kClaimed = 1ull << 62;  // LDS key word: key_hi | kClaimed, then | kReady (key_hi < 2^58)
constexpr uint64_t kReady = 1ull << 63;
constexpr uint32_t kLdsSpin = 1u << 20;    // bound on waiting for another wave's claim to be published

struct CountArgs {
    const uint4 *recs;
    const uint64_t *bin_start;
    uint64_t n_bins;
    uint64_t seed;
    uint32_t min_depth, ext_min;
    uint32_t bypass;
    uint32_t uu_only;
    uint32_t *status;
    unsigned long long *stats;
    uint4 *stage;  // kCountGrid areas of kStage records, 4 x 16 bytes each
};

struct BinLds {
    uint64_t hi[kBinSlots];      // 0 = empty; key_hi | kClaimed while the second word is written; | kReady after
    uint64_t lo[kBinSlots];
    uint32_t cnt[9][kBinSlots];  // no left extension, left A..T, right A..T
    uint32_t bloom[kBloomWords];
    uint32_t defer[kDeferCap];   // bin-relative record index of each deferred occurrence
    uint32_t n_defer, n_keys, spill, staged;
    uint32_t wsum[kBlock / 64];
    unsigned long long base;
};

// Hash of a key inside its bin (home slot in the low 9 bits, filter word in the next 9, filter
// bits in the top 20): a multilinear sum of the key's four 32-bit words mod 2^32, then a
// xorshift-multiply mix.  The bin itself was chosen by another hash, so any good mix of the
// key works here; the output does not depend on it.
__device__ __forceinline__ uint32_t bin_local_hash(uint64_t hi, uint64_t lo, uint32_t seed) {
    uint32_t x = seed + (uint32_t)lo * 0x9E3779B1u + (uint32_t)(lo >> 32) * 0x85EBCA77u + (uint32_t)hi * 0xC2B2AE3Du +
                 (uint32_t)(hi >> 32) * 0x27D4EB2Fu;
    x ^= x >> 15;
    x *= 0x2C1B3C6Du;
    x ^= x >> 13;
    return x;
}

__device__ __forceinline__ uint64_t lds_word(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until a claimed slot's key is published (x: its first word as read); false past the bound.
__device__ __forceinline__ bool lds_published(const BinLds &t, uint32_t s, uint64_t &x) {
    for (uint32_t spins = 0; !(x & kReady); ++spins) {
        if (spins > kLdsSpin) return false;
        x = lds_word(&t.hi[s]);
    }
    return true;
}

// Slot of the key in the bin's table: -1 absent, -2 a claim stayed unpublished past the bound.
// Only another wave can hold a claim unpublished here (a wave publishes its own claims before
// it looks up its next occurrences).
__device__ __forceinline__ int lds_find(const BinLds &t, uint64_t hi, uint64_t lo, uint32_t h) {
    const uint64_t want = hi | kClaimed;
    uint32_t s = h & (kBinSlots - 1);
    for (int p = 0; p < kBinSlots; ++p) {
        uint64_t x = lds_word(&t.hi[s]);
        if (x == 0) return -1;
        if ((x & ~kReady) == want) {
            if (!lds_published(t, s, x)) return -2;
            if (t.lo[s] == lo) return (int)s;
        }
        s = (s + 1) & (kBinSlots - 1);
    }
    return -1;
}

// Insert the key of every lane with `act` (or find it, if another lane got there first) and
// return its slot; -2 when the probe met no free slot or a claim stayed unpublished.  Called by
// every lane of the wave.  A lane claims an empty slot with a compare-and-swap of the first
// word to key_hi | kClaimed, stores the second word and sets kReady; the claims of one step are
// published before any lane of the wave compares a claimed slot's key, so a wave never waits
// for itself, and lanes of other waves wait for kReady.
__device__ __forceinline__ int lds_insert(BinLds &t, bool act, uint64_t hi, uint64_t lo, uint32_t h, bool &added) {
    const uint64_t want = hi | kClaimed;
    uint32_t s = h & (kBinSlots - 1), probes = 0;
    int res = -2;
    bool active = act;
    added = false;
    while (__ballot(active)) {
        bool won = false;
        uint64_t x = 0;
        if (active) {
            x = lds_word(&t.hi[s]);
            if (x == 0) {
                unsigned long long e = 0;
                won = __hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(&t.hi[s]), &e,
                                                           (unsigned long long)want, __ATOMIC_ACQ_REL,
                                                           __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
                x = won ? want : e;
            }
        }
        if (won) {
            t.lo[s] = lo;
            __hip_atomic_fetch_or(reinterpret_cast<unsigned long long *>(&t.hi[s]), (unsigned long long)kReady,
                                  __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (active) {
            if (won) {
                res = (int)s;
                added = true;
                active = false;
            } else {
                if ((x & ~kReady) == want) {
                    if (!lds_published(t, s, x)) {
                        active = false;
                    } else if (t.lo[s] == lo) {
                        res = (int)s;
                        active = false;
                    }
                }
                if (active) {
                    s = (s + 1) & (kBinSlots - 1);
                    if (++probes >= (uint32_t)kBinSlots) active = false;
                }
            }
        }
    }
    return res;
}

__device__ __forceinline__ void lds_count(BinLds &t, int s, int left, int right) {
    atomicAdd(&t.cnt[left < 4 ? 1 + left : 0][s], 1u);
    if (right < 4) atomicAdd(&t.cnt[5 + right][s], 1u);
}

// Filter word and bits of a key in its bin's Bloom filter: 4 bits of one 32-bit word, from bits
// of the in-bin hash other than those of the home slot.
__device__ __forceinline__ void lds_bloom_bits(uint32_t h, uint32_t &w, uint32_t &m) {
    w = (h >> 9) & (kBloomWords - 1);
    m = (1u << ((h >> 12) & 31)) | (1u << ((h >> 17) & 31)) | (1u << ((h >> 22) & 31)) | (1u << (h >> 27));
}

// Move the workgroup's staged records to the export (one atomic add takes their range).  Called
// by every thread of the workgroup.
__device__ __forceinline__ void stage_flush(BinLds &t, const uint4 *area, const hm_export_t &out, uint32_t *status) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the staged stores are in L2
    __syncthreads();
    const uint32_t n = t.staged;
    if (threadIdx.x == 0 && n)
        t.base = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_out), (unsigned long long)n);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // read them from L2, not a stale L1 line
    const uint64_t base = t.base;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        const uint4 q0 = area[4 * i], q1 = area[4 * i + 1], q2 = area[4 * i + 2], q3 = area[4 * i + 3];
        const uint64_t idx = base + i;
        if (idx < out.capacity) {
            out.key_lo[idx] = ((uint64_t)q0.y << 32) | q0.x;
            out.key_hi[idx] = ((uint64_t)q0.w << 32) | q0.z;
            *reinterpret_cast<uint4 *>(out.tl + 4 * idx) = q1;
            *reinterpret_cast<uint4 *>(out.tr + 4 * idx) = q2;
            out.count[idx] = q3.x;
            out.cls_l[idx] = (uint8_t)q3.y;
            out.cls_r[idx] = (uint8_t)(q3.y >> 8);
        } else {
            atomicOr(status, HM_ST_OUTPUT_FULL);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) t.staged = 0;
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_count_bins(CountArgs c, hm_export_t out, hm_occ_t spill) {
    __shared__ BinLds t;
    const uint32_t lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint4 *area = c.stage + (size_t)blockIdx.x * kStage * 4;
    auto clear = [&]() {
        for (int i = threadIdx.x; i < kBinSlots; i += kBlock) t.hi[i] = 0;
        uint4 *cz = reinterpret_cast<uint4 *>(&t.cnt[0][0]);
        for (int i = threadIdx.x; i < 9 * kBinSlots / 4; i += kBlock) cz[i] = make_uint4(0, 0, 0, 0);
        uint4 *bz = reinterpret_cast<uint4 *>(t.bloom);
        for (int i = threadIdx.x; i < kBloomWords / 4; i += kBlock) bz[i] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) t.n_defer = t.n_keys = t.spill = 0;
    };
    clear();
    if (threadIdx.x == 0) t.staged = 0;
    __syncthreads();
    uint64_t dsum = 0, dxor = 0;
    uint64_t st_recs = 0, st_spilled_bins = 0, st_spilled = 0, st_defer = 0, st_keys = 0, st_kept = 0;
    for (uint64_t bin = blockIdx.x; bin < c.n_bins; bin += gridDim.x) {
        const uint64_t b0 = c.bin_start[bin];
        const uint64_t n = c.bin_start[bin + 1] - b0;  // workgroup-uniform
        if (n == 0) continue;
        const uint4 *R = c.recs + b0;
        uint64_t bin_recs = 0;  // this thread's records of the bin (holes aside)
        // one pass over the bin's occurrences: count, or test the filter and insert, or defer
        // the next round's records are loaded while this round's are counted
        uint4 nxt[kCPer];
#pragma unroll
        for (int j = 0; j < kCPer; ++j) {
            const uint64_t i = (uint64_t)j * kBlock + threadIdx.x;
            nxt[j] = i < n ? R[i] : make_uint4(0, 0, 0, 0);
        }
        for (uint64_t c0 = 0; c0 < n; c0 += kCChunk) {
            if (t.spill) break;  // set by any wave; the other waves may finish their round
            uint4 r[kCPer];
#pragma unroll
            for (int j = 0; j < kCPer; ++j) {
                r[j] = nxt[j];
                const uint64_t i = c0 + kCChunk + j * kBlock + threadIdx.x;
                nxt[j] = i < n ? R[i] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < kCPer; ++j) {
                const uint64_t i = c0 + j * kBlock + threadIdx.x;
                const bool valid = i < n && !is_hole(r[j]);
                bin_recs += valid ? 1 : 0;
                const Rec x = rec_unpack(r[j]);
                const uint32_t h = valid ? bin_local_hash(x.hi, x.lo, (uint32_t)c.seed) : 0u;
                const int s = valid ? lds_find(t, x.hi, x.lo, h) : -1;
                bool ins = false;
                if (s >= 0) {
                    lds_count(t, s, x.left, x.right);
                } else if (s == -2) {
                    t.spill = 1;
                } else if (valid) {
                    ins = c.bypass != 0;
                    if (!ins) {
                        uint32_t w, m;
                        lds_bloom_bits(h, w, m);
                        ins = (atomicOr(&t.bloom[w], m) & m) == m;
                    }
                }
                // deferred: one LDS atomic per wave reserves the wave's entries
                const bool dfr = valid && s == -1 && !ins;
                const uint64_t dm = __ballot(dfr);
                if (dm) {
                    const int leader = __ffsll((long long)dm) - 1;
                    uint32_t d0 = 0;
                    if ((int)lane == leader) d0 = atomicAdd(&t.n_defer, (uint32_t)__popcll(dm));
                    d0 = __shfl(d0, leader);
                    if (dfr) {
                        const uint32_t d = d0 + lanes_below(dm);
                        if (d < (uint32_t)kDeferCap) t.defer[d] = (uint32_t)i;
                        else t.spill = 1;
                    }
                }
                bool added;
                const int si = lds_insert(t, ins, x.hi, x.lo, h, added);
                if (ins) {
                    if (si >= 0) lds_count(t, si, x.left, x.right);
                    else t.spill = 1;
                }
                if (added && atomicAdd(&t.n_keys, 1u) >= kMaxKeys) t.spill = 1;
            }
        }
        __syncthreads();
        if (!t.spill) {
            st_recs += bin_recs;
            // deferred occurrences: counted when their k-mer is in the table
            const uint32_t nd = t.n_defer;
            for (uint32_t d = threadIdx.x; d < nd; d += kBlock) {
                const Rec x = rec_unpack(R[t.defer[d]]);
                const int s = lds_find(t, x.hi, x.lo, bin_local_hash(x.hi, x.lo, (uint32_t)c.seed));
                if (s >= 0) lds_count(t, s, x.left, x.right);
            }
            if (threadIdx.x == 0) {
                st_defer += nd;
                st_keys += t.n_keys;
            }
            __syncthreads();
            // depth filter, classification and export of the bin's table (two slots a thread),
            // staged in the workgroup's area
            bool take[2];
            uint32_t tl[2][4], tr[2][4], count[2], cl[2], cr[2];
            uint64_t khi[2], klo[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int s = j * kBlock + threadIdx.x;
                const uint64_t th = t.hi[s];
                take[j] = false;
                count[j] = cl[j] = cr[j] = 0;
                khi[j] = th & ((1ull << kExtShift) - 1);
                klo[j] = 0;
                if (th) {
                    uint64_t cnt = t.cnt[0][s];
                    for (int q = 0; q < 4; ++q) {
                        tl[j][q] = t.cnt[1 + q][s];
                        tr[j][q] = t.cnt[5 + q][s];
                        cnt += tl[j][q];
                    }
                    count[j] = (uint32_t)cnt;
                    cl[j] = side_class(tl[j], c.ext_min);
                    cr[j] = side_class(tr[j], c.ext_min);
                    take[j] = cnt >= c.min_depth && (!c.uu_only || (cl[j] < 4 && cr[j] < 4));
                    klo[j] = t.lo[s];
                }
            }
            const uint64_t m0 = __ballot(take[0]), m1 = __ballot(take[1]);
            if (lane == 0) t.wsum[wave] = (uint32_t)(__popcll(m0) + __popcll(m1));
            __syncthreads();
            uint32_t tot = 0, before = 0;
            for (int q = 0; q < kBlock / 64; ++q) {
                before += q < wave ? t.wsum[q] : 0u;
                tot += t.wsum[q];
            }
            if (t.staged + tot > (uint32_t)kStage) stage_flush(t, area, out, c.status);  // uniform
            const uint32_t at = t.staged + before;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!take[j]) continue;
                const uint32_t i = at + (j == 0 ? lanes_below(m0) : (uint32_t)__popcll(m0) + lanes_below(m1));
                area[4 * i] = make_uint4((uint32_t)klo[j], (uint32_t)(klo[j] >> 32), (uint32_t)khi[j],
                                         (uint32_t)(khi[j] >> 32));
                area[4 * i + 1] = make_uint4(tl[j][0], tl[j][1], tl[j][2], tl[j][3]);
                area[4 * i + 2] = make_uint4(tr[j][0], tr[j][1], tr[j][2], tr[j][3]);
                area[4 * i + 3] = make_uint4(count[j], cl[j] | (cr[j] << 8), 0u, 0u);
                if (out.digest) {
                    const uint64_t y = record_hash(khi[j], klo[j], count[j], tl[j], tr[j], cl[j], cr[j]);
                    dsum += y;
                    dxor ^= y;
                }
                ++st_kept;
            }
            __syncthreads();
            if (threadIdx.x == 0) t.staged += tot;
        } else {
            // the bin goes to the global-table path whole
            if (threadIdx.x == 0) {
                t.base = atomicAdd(reinterpret_cast<unsigned long long *>(spill.count), (unsigned long long)n);
                st_spilled_bins += 1;
            }
            __syncthreads();
            const uint64_t base = t.base;
            for (uint64_t i = threadIdx.x; i < n; i += kBlock) {
                const uint4 rr = R[i];
                const Rec x = rec_unpack(rr);
                const uint64_t idx = base + i;
                if (idx < spill.capacity) {
                    *reinterpret_cast<uint4 *>(spill.keys + 2 * idx) =
                        make_uint4((uint32_t)x.hi, (uint32_t)(x.hi >> 32), (uint32_t)x.lo, (uint32_t)(x.lo >> 32));
                    spill.ext[idx] = is_hole(rr) ? kHole : (uint8_t)(x.left | (x.right << 4));
                    st_spilled += is_hole(rr) ? 0 : 1;
                    st_recs += is_hole(rr) ? 0 : 1;
                } else {
                    atomicOr(c.status, HM_ST_STREAM_FULL);
                }
            }
        }
        __syncthreads();
        clear();
        __syncthreads();
    }
    stage_flush(t, area, out, c.status);
    digest_flush(out, dsum, dxor);
    if (c.stats) {
        const uint64_t v[6] = {st_recs, st_spilled_bins, st_spilled, st_defer, st_keys, st_kept};
        for (int q = 0; q < 6; ++q) {
            uint64_t x = v[q];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            if (lane == 0 && x) atomicAdd(c.stats + q, (unsigned long long)x);
        }
    }
}

// ------------------------------------------------------------------ merging two exports

// Append src's records [0, *src.n_out) to dst after its *dst.n_out records.  The counts are read
// before any thread moves them (k_merge_counts runs after this kernel).
__global__ __launch_bounds__(kBlock) void k_merge_copy(hm_export_t src, hm_export_t dst, uint32_t *status) {
    const uint64_t ns = min(*src.n_out, src.capacity), nd = *dst.n_out;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < ns; i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t j = nd + i;
        if (j >= dst.capacity) {
            atomicOr(status, HM_ST_OUTPUT_FULL);
            continue;
        }
        dst.key_hi[j] = src.key_hi[i];
        dst.key_lo[j] = src.key_lo[i];
        dst.count[j] = src.count[i];
        *reinterpret_cast<uint4 *>(dst.tl + 4 * j) = *reinterpret_cast<const uint4 *>(src.tl + 4 * i);
        *reinterpret_cast<uint4 *>(dst.tr + 4 * j) = *reinterpret_cast<const uint4 *>(src.tr + 4 * i);
        dst.cls_l[j] = src.cls_l[i];
        dst.cls_r[j] = src.cls_r[i];
    }
}

__global__ void k_merge_counts(hm_export_t src, hm_export_t dst, uint32_t *status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (*src.n_out > src.capacity) *status |= HM_ST_OUTPUT_FULL;  // src was already short
    *dst.n_out += *src.n_out;
    if (dst.digest && src.digest) {
        dst.digest[0] += src.digest[0];
        dst.digest[1] ^= src.digest[1];
    }
}


// scratch layout: the staging areas of hm_count_bins (kCountGrid x kStage records of 64 bytes),
// then the group starts in tmp and in recs (ng + 1 words each), the group totals (ng words
// each) and the two histograms (32-bit counters)
constexpr uint64_t kStageBytes = (uint64_t)kCountGrid * kStage * 64;

struct Scratch {
    uint4 *stage;
    uint64_t *wstart, *wtot, *gstart2, *gtot2;
    uint32_t *hist1, *hist2;
};

Scratch scratch_of(const hm_bins_t *b) {
    const uint64_t ng = 1ull << b->group_bits;
    Scratch s;
    s.stage = reinterpret_cast<uint4 *>(b->scratch);
    s.wstart = b->scratch + kStageBytes / 8;
    s.wtot = s.wstart + kGrid1 + 1;
    s.gstart2 = s.wtot + kGrid1;
    s.gtot2 = s.gstart2 + ng + 1;
    s.hist1 = reinterpret_cast<uint32_t *>(s.gtot2 + ng);
    s.hist2 = s.hist1 + ng * kGrid1;
    return s;
}

// records hm_bin_kmers needs room for: the windows plus the padding of both levels' ranges
// dynamic LDS of the first-level scatter for ng groups: the combiner and the range starts
size_t scatter1_lds(size_t ng) { return Combiner<kBlk1>::bytes(ng) + 4 * ng; }
constexpr size_t kScatter1StaticLds = 8 * (kTileB2Words + 2 * kTileMaskWords);  // the staged tile
constexpr size_t kLdsPerCu = 160 * 1024;

uint64_t bins_capacity(uint64_t windows, uint32_t group_bits, uint32_t bin_bits, uint64_t g1) {
    const uint64_t ng = 1ull << group_bits, nb = 1ull << (group_bits + bin_bits);
    const uint64_t pad1 = (uint64_t)(kBlk1 - 1) * g1 * ng, pad2 = (uint64_t)(kBlk2 - 1) * nb * kSlices;
    return windows + (pad1 > pad2 ? pad1 : pad2);
}

}  // namespace

int check_bins(const hm_bins_t *b) {
    if (!b || !b->recs || !b->tmp || !b->scratch || !b->bin_start || !b->status)
        return fail(HM_EINVAL, "bins: a buffer is NULL");
    if (((uintptr_t)b->recs) & 127 || ((uintptr_t)b->tmp) & 127 || ((uintptr_t)b->scratch) & 15)
        return fail(HM_EINVAL, "bins: recs and tmp must be 128-byte aligned, scratch 16-byte aligned");
    if (b->group_bits > (uint32_t)kMaxGroupBits || b->bin_bits > (uint32_t)kMaxBinBits)
        return fail(HM_EINVAL, "bins: group_bits must be at most %d and bin_bits at most %d", kMaxGroupBits,
                    kMaxBinBits);
    return HM_OK;
}

int bins_grid1(int64_t n_tiles, uint32_t group_bits) {
    // as many workgroups as the first-level scatter's LDS lets a CU hold at once
    const size_t per_wg = scatter1_lds((size_t)1 << group_bits) + kScatter1StaticLds;
    const int64_t per_cu = (int64_t)(kLdsPerCu / per_wg);
    int64_t cap = (per_cu > 0 ? per_cu : 1) * (int64_t)device_cus();
    if (cap > kGrid1) cap = kGrid1;
    return (int)(n_tiles < cap ? n_tiles : cap);
}

uint32_t *bins_hist1(const hm_bins_t *b) { return scratch_of(b).hist1; }

namespace {
// What a first-level histogram in a bins scratch was counted for, noted by hm_cardinality_bins
// and taken (whatever the flags) by the next hm_bin_kmers on that scratch: a histogram of other
// reads, parameters or bin counts would send the scatter's records outside their ranges.
struct Counted {
    const void *bases2;
    int64_t n_reads;
    int32_t read_len, k, forward_only;
    uint32_t n_owners, owner, group_bits, bin_bits;
    int device;
    bool operator==(const Counted &o) const {
        return bases2 == o.bases2 && n_reads == o.n_reads && read_len == o.read_len && k == o.k &&
               forward_only == o.forward_only && n_owners == o.n_owners && owner == o.owner &&
               group_bits == o.group_bits && bin_bits == o.bin_bits && device == o.device;
    }
};

Counted counted_key(const hm_bins_t *b, const hm_reads_t *r, const hm_params_t *p) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    return Counted{r->bases2, r->n_reads, r->read_len, p->k, (p->flags & HM_FORWARD_ONLY) ? 1 : 0,
                   p->n_owners, p->owner, b->group_bits, b->bin_bits, dev};
}

std::mutex g_counted_mu;
std::unordered_map<const void *, Counted> g_counted;  // by scratch address
}  // namespace

void bins_note_counted(const hm_bins_t *b, const hm_reads_t *r, const hm_params_t *p) {
    const Counted c = counted_key(b, r, p);
    std::lock_guard<std::mutex> g(g_counted_mu);
    g_counted[b->scratch] = c;
}

bool bins_take_counted(const hm_bins_t *b, const hm_reads_t *r, const hm_params_t *p) {
    const Counted c = counted_key(b, r, p);
    std::lock_guard<std::mutex> g(g_counted_mu);
    auto it = g_counted.find(b->scratch);
    if (it == g_counted.end()) return false;
    const bool same = it->second == c;
    g_counted.erase(it);
    return same;
}

void bins_drop_counted(const hm_bins_t *b) {
    std::lock_guard<std::mutex> g(g_counted_mu);
    g_counted.erase(b->scratch);
}

}  // namespace hm

using namespace hm;

extern "C" {

size_t hm_bins_scratch_bytes(uint32_t group_bits, uint32_t bin_bits) {
    if (group_bits > (uint32_t)kMaxGroupBits || bin_bits > (uint32_t)kMaxBinBits) return 0;
    const uint64_t ng = 1ull << group_bits, nb = 1ull << (group_bits + bin_bits);
    return (size_t)(kStageBytes + 8 * (2 * kGrid1 + 2 * ng + 2) + 4 * ng * kGrid1 + 4 * nb * kSlices);
}

uint64_t hm_bins_capacity(uint64_t windows, uint32_t group_bits, uint32_t bin_bits) {
    if (group_bits > (uint32_t)kMaxGroupBits || bin_bits > (uint32_t)kMaxBinBits) return 0;
    return bins_capacity(windows, group_bits, bin_bits, kGrid1);
}

namespace {
// the first level's regions: each workgroup's pieces (a row of hist1, rounded up to blocks), then
// the regions one after the other
void level1_regions(const Scratch &sc, int g1, int ng, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)g1), dim3(kBlock), 0, s, sc.hist1, ng, (uint32_t)kBlk1, sc.wtot);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, s, sc.wtot, g1, sc.wstart);
}

// the second level, from the first level's pieces in b->tmp to the bins in b->recs
void level2(const hm_bins_t *b, const Scratch &sc, int g1, int total_bits, int bin_bits, hipStream_t s) {
    const uint64_t ng = 1ull << (total_bits - bin_bits), ns = 1ull << bin_bits, n_bins = 1ull << total_bits;
    const uint4 *tmp = reinterpret_cast<const uint4 *>(b->tmp);
    uint4 *recs = reinterpret_cast<uint4 *>(b->recs);
    const size_t lds2 = Combiner<kBlk2>::bytes(ns) + 4 * ns;  // the combiner and the range starts
    const dim3 g2((unsigned)(ng * kSlices));
    hipLaunchKernelGGL(k_hist2, g2, dim3(kBlock), ns * 4, s, tmp, sc.hist1, sc.wstart, g1, sc.hist2, total_bits,
                       bin_bits);
    hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)ng), dim3(kBlock), 0, s, sc.hist2, (int)(ns * kSlices),
                       (uint32_t)kBlk2, sc.gtot2);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, s, sc.gtot2, (int)ng, sc.gstart2);
    hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)grid_for(n_bins + 1, 16)), dim3(kBlock), 0, s, sc.hist2,
                       sc.gstart2, b->bin_start, total_bits, bin_bits);
    hipLaunchKernelGGL(k_scatter2, g2, dim3(kT2), lds2, s, tmp, sc.hist1, sc.wstart, g1, sc.gstart2, sc.hist2, recs,
                       total_bits, bin_bits);
}
}  // namespace

int hm_bin_kmers(const hm_reads_t *r, const hm_params_t *p, hm_bins_t *b, uint32_t flags, hipStream_t s) {
    if (flags & ~HM_BINS_COUNTED) return fail(HM_EINVAL, "hm_bin_kmers: unknown flags 0x%x", flags);
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_reads(r, p->k);
    if (rc) return rc;
    rc = check_bins(b);
    if (rc) return rc;
    if (p->k > kMaxBinK) return fail(HM_EINVAL, "binned counting needs k <= %d (k=%d)", kMaxBinK, p->k);
    if (r->n_reads > 0 && r->read_off) return fail(HM_EINVAL, "binned counting needs fixed-length reads (read_off NULL)");
    if (r->n_reads > 0 && r->read_len > kTileBases - 64)
        return fail(HM_EINVAL, "binned counting needs reads of at most %d bases", kTileBases - 64);
    const int total_bits = (int)(b->group_bits + b->bin_bits), bin_bits = (int)b->bin_bits;
    const uint64_t ng = 1ull << b->group_bits, n_bins = 1ull << total_bits;
    const int64_t W = r->n_reads > 0 ? (int64_t)r->read_len - p->k + 1 : 0;
    const uint64_t windows = W > 0 ? (uint64_t)r->n_reads * (uint64_t)W : 0;
    if (bins_capacity(windows, b->group_bits, b->bin_bits, kGrid1) >= (1ull << 32))
        return fail(HM_EINVAL, "binned counting takes fewer than 2^32 records (windows and padding) per call");
    const int32_t rpt = windows ? kTileBases / r->read_len : 1;
    const int64_t n_tiles = windows ? (r->n_reads + rpt - 1) / rpt : 0;
    const int g1 = bins_grid1(n_tiles, b->group_bits);
    if (bins_capacity(windows, b->group_bits, b->bin_bits, (uint64_t)g1) > b->capacity)
        return fail(HM_EINVAL, "bins hold %llu records, the reads need %llu (windows and padding; see hm_bins_capacity)",
                    (unsigned long long)b->capacity,
                    (unsigned long long)bins_capacity(windows, b->group_bits, b->bin_bits, (uint64_t)g1));
    if (!bins_take_counted(b, r, p) && (flags & HM_BINS_COUNTED))
        return fail(HM_EINVAL, "hm_bin_kmers: HM_BINS_COUNTED, but the last hm_cardinality_bins on these bins' scratch "
                    "was not over the same reads, params and bin counts (or a partition has used its histogram)");
    rc = fill<uint32_t>(b->status, 1, 0u, s);
    if (rc) return rc;
    if (b->stats) {
        rc = fill<uint64_t>(b->stats, HM_N_BIN_STATS, 0ull, s);
        if (rc) return rc;
    }
    if (windows == 0) return fill<uint64_t>(b->bin_start, n_bins + 1, 0ull, s);
    const Scratch sc = scratch_of(b);
    PassArgs a;
    memset(&a, 0, sizeof a);
    a.b2 = r->bases2;
    a.nm = r->nmask;
    a.hq = r->hqmask;
    a.n_reads = r->n_reads;
    a.n_bases = r->n_bases;
    a.read_len = r->read_len;
    a.k = p->k;
    a.forward_only = (p->flags & HM_FORWARD_ONLY) ? 1 : 0;
    a.n_owners = p->n_owners;
    a.owner = p->owner;
    a.seed = p->seed;
    a.status = b->status;
    uint4 *tmp = reinterpret_cast<uint4 *>(b->tmp);
    const size_t lds1 = scatter1_lds(ng);  // the combiner's arrays and the range starts
    const bool two = p->k >= 32;           // keys of two 64-bit words
    if (!(flags & HM_BINS_COUNTED))  // else hm_cardinality_bins counted the histogram on its way
        hipLaunchKernelGGL(two ? k_hist1<2> : k_hist1<1>, dim3(g1), dim3(kBlock), ng * 4, s, a, rpt, n_tiles,
                           sc.hist1, total_bits, bin_bits);
    level1_regions(sc, g1, (int)ng, s);
    hipLaunchKernelGGL(two ? k_scatter1<2> : k_scatter1<1>, dim3(g1), dim3(kT1), lds1, s, a, rpt, n_tiles,
                       sc.hist1, sc.wstart, tmp, total_bits, bin_bits);
    level2(b, sc, g1, total_bits, bin_bits, s);
    HM_LAUNCH_CHECK("hm_bin_kmers");
    return HM_OK;
}

int hm_bin_occ(const hm_occ_t *o, const hm_params_t *p, hm_bins_t *b, hipStream_t s) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_occ(o);
    if (rc) return rc;
    rc = check_bins(b);
    if (rc) return rc;
    if (p->k > kMaxBinK) return fail(HM_EINVAL, "binned counting needs k <= %d (k=%d)", kMaxBinK, p->k);
    const int total_bits = (int)(b->group_bits + b->bin_bits), bin_bits = (int)b->bin_bits;
    const uint64_t ng = 1ull << b->group_bits, n_bins = 1ull << total_bits;
    // the stream's entries are at most its capacity; the grid is the one the first level's LDS allows
    if (bins_capacity(o->capacity, b->group_bits, b->bin_bits, kGrid1) >= (1ull << 32))
        return fail(HM_EINVAL, "binned counting takes fewer than 2^32 records (stream capacity and padding) per call");
    const int g1 = bins_grid1(kGrid1, b->group_bits);
    if (bins_capacity(o->capacity, b->group_bits, b->bin_bits, (uint64_t)g1) > b->capacity)
        return fail(HM_EINVAL, "bins hold %llu records, a stream of %llu entries needs %llu (see hm_bins_capacity)",
                    (unsigned long long)b->capacity, (unsigned long long)o->capacity,
                    (unsigned long long)bins_capacity(o->capacity, b->group_bits, b->bin_bits, (uint64_t)g1));
    bins_drop_counted(b);  // a histogram noted for these bins is not this partition's
    rc = fill<uint32_t>(b->status, 1, 0u, s);
    if (rc) return rc;
    if (b->stats) {
        rc = fill<uint64_t>(b->stats, HM_N_BIN_STATS, 0ull, s);
        if (rc) return rc;
    }
    if (o->capacity == 0) return fill<uint64_t>(b->bin_start, n_bins + 1, 0ull, s);
    const Scratch sc = scratch_of(b);
    uint4 *tmp = reinterpret_cast<uint4 *>(b->tmp);
    hipLaunchKernelGGL(k_hist1_occ, dim3(g1), dim3(kHistT), ng * 4, s, *o, sc.hist1, total_bits, bin_bits);
    level1_regions(sc, g1, (int)ng, s);
    hipLaunchKernelGGL(k_scatter1_occ, dim3(g1), dim3(kT1), scatter1_lds(ng), s, *o, sc.hist1, sc.wstart, tmp,
                       total_bits, bin_bits);
    level2(b, sc, g1, total_bits, bin_bits, s);
    HM_LAUNCH_CHECK("hm_bin_occ");
    return HM_OK;
}

int hm_count_bins(const hm_bins_t *b, const hm_params_t *p, uint32_t flags, hm_export_t *out, hm_occ_t *spill,
                  hipStream_t s) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_bins(b);
    if (rc) return rc;
    if (p->k > kMaxBinK) return fail(HM_EINVAL, "binned counting needs k <= %d (k=%d)", kMaxBinK, p->k);
    if (flags & ~HM_EXPORT_UU_ONLY) return fail(HM_EINVAL, "hm_count_bins: only HM_EXPORT_UU_ONLY may be set");
    if (!out || !out->n_out) return fail(HM_EINVAL, "export: out or n_out is NULL");
    if (out->capacity > 0 && (!out->key_hi || !out->key_lo || !out->count || !out->tl || !out->tr || !out->cls_l ||
                              !out->cls_r))
        return fail(HM_EINVAL, "export arrays are NULL");
    if ((((uintptr_t)out->tl) | ((uintptr_t)out->tr)) & 15) return fail(HM_EINVAL, "export tl/tr must be 16-byte aligned");
    rc = check_occ(spill);
    if (rc) return rc;
    rc = fill<uint64_t>(out->n_out, 1, 0ull, s);
    if (!rc && out->digest) rc = fill<uint64_t>(out->digest, 2, 0ull, s);
    if (!rc) rc = fill<uint64_t>(spill->count, 1, 0ull, s);
    if (rc) return rc;
    CountArgs c;
    c.recs = reinterpret_cast<const uint4 *>(b->recs);
    c.bin_start = b->bin_start;
    c.n_bins = 1ull << (b->group_bits + b->bin_bits);
    c.seed = p->seed;
    c.min_depth = p->min_depth;
    c.ext_min = p->ext_min;
    c.bypass = ((p->flags & HM_BLOOM_BYPASS) || p->min_depth == 1) ? 1 : 0;
    c.uu_only = (flags & HM_EXPORT_UU_ONLY) ? 1 : 0;
    c.status = b->status;
    c.stats = reinterpret_cast<unsigned long long *>(b->stats);
    c.stage = scratch_of(b).stage;
    uint64_t cap = (uint64_t)device_cus() * kCountBlocksPerCu;
    if (cap > (uint64_t)kCountGrid) cap = kCountGrid;
    const dim3 g((unsigned)(c.n_bins < cap ? c.n_bins : cap));
    hipLaunchKernelGGL(k_count_bins, g, dim3(kBlock), 0, s, c, *out, *spill);
    HM_LAUNCH_CHECK("hm_count_bins");
    return HM_OK;
}

int hm_export_merge(const hm_export_t *src, hm_export_t *dst, uint32_t *status, hipStream_t s) {
    if (!src || !dst || !src->n_out || !dst->n_out || !status) return fail(HM_EINVAL, "merge: an argument is NULL");
    if ((((uintptr_t)src->tl) | ((uintptr_t)src->tr) | ((uintptr_t)dst->tl) | ((uintptr_t)dst->tr)) & 15)
        return fail(HM_EINVAL, "merge: tl/tr must be 16-byte aligned");
    const uint64_t g = grid_for(src->capacity > 0 ? src->capacity : 1, 8);
    hipLaunchKernelGGL(k_merge_copy, dim3((unsigned)g), dim3(kBlock), 0, s, *src, *dst, status);
    hipLaunchKernelGGL(k_merge_counts, dim3(1), dim3(64), 0, s, *src, *dst, status);
    HM_LAUNCH_CHECK("hm_export_merge");
    return HM_OK;
}

}  // extern "C"
