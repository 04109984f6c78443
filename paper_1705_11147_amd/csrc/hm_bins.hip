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
#include "hm_device.h"

namespace hm {
namespace {

// bin map: multiply-shift hashing (any odd constants; the output does not depend on them)
constexpr uint64_t kBinMul1 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kBinMul2 = 0x165667B19E3779F9ull;
constexpr int kGrid1 = 1024;       // most workgroups of the two passes over the reads
constexpr int kSlices = 8;         // workgroups per group in the second partition level
constexpr int kMaxBits = 12;       // group_bits and bin_bits are each at most this
constexpr int kBinSlots = 512;     // LDS table of one bin
constexpr int kBloomWords = 512;   // 32-bit filter words: 16384 bits per bin
constexpr int kDeferCap = 2048;    // deferred occurrences of one bin
constexpr int kPer = 4;            // records per thread per round
constexpr int kChunk = kPer * kBlock;
constexpr uint32_t kMaxKeys = kBinSlots * 3 / 4;
constexpr uint64_t kTaken = 1ull << 63;  // marks an occupied LDS slot (key_hi < 2^58)
constexpr int kExtShift = 58;
constexpr int kMaxBinK = 61;       // 2k + 6 extension bits fit in 128
constexpr int kCountBlocksPerCu = 4;

__device__ __forceinline__ uint64_t bin_hash(uint64_t hi, uint64_t lo) { return (lo ^ hi * kBinMul1) * kBinMul2; }

// bin of a key: the top `bits` bits of its bin hash (0 when bits == 0)
__device__ __forceinline__ uint32_t bin_of(uint64_t hi, uint64_t lo, int bits) {
    return bits ? (uint32_t)(bin_hash(hi, lo) >> (64 - bits)) : 0u;
}

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

// Level-1 histogram: counts of each group's windows in this workgroup's tiles (the tiles
// fixed_windows hands a workgroup depend only on the grid, which the scatter pass repeats).
__global__ __launch_bounds__(kBlock) void k_hist1(PassArgs a, int32_t rpt, int64_t n_tiles, uint32_t *hist1,
                                                  int total_bits, int bin_bits) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    extern __shared__ uint32_t s_h[];
    const int ng = 1 << (total_bits - bin_bits);
    for (int i = threadIdx.x; i < ng; i += kBlock) s_h[i] = 0;
    fixed_windows<false>(a, rpt, n_tiles, s_b2, s_nm, s_hq, [&](bool act, const Occ &o, int64_t) {
        if (act) atomicAdd(&s_h[bin_of(o.hi, o.lo, total_bits) >> bin_bits], 1u);
    });
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += kBlock) hist1[(size_t)i * gridDim.x + blockIdx.x] = s_h[i];
}

// Exclusive prefix sum of each row of x (rows x cols, one workgroup per row) in place; the row
// total to tot[row] when tot is not NULL.  Every row total is below 2^32 (checked by the host).
__global__ __launch_bounds__(kBlock) void k_scan_rows(uint32_t *x, int cols, uint64_t *tot) {
    __shared__ uint32_t s_part[kBlock];
    uint32_t *row = x + (size_t)blockIdx.x * cols;
    const int per = (cols + kBlock - 1) / kBlock;
    const int b = min((int)threadIdx.x * per, cols), e = min(b + per, cols);
    uint32_t sum = 0;
    for (int i = b; i < e; ++i) sum += row[i];
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
        const uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (tot && threadIdx.x == kBlock - 1) tot[blockIdx.x] = s_part[kBlock - 1];
}

// start[g] = sum of tot[0..g), g = 0..n (one workgroup, n <= 2^kMaxBits)
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

// Level-1 scatter: the same windows as k_hist1, each written to its group's range at the
// workgroup's offset (an LDS cursor per group).
__global__ __launch_bounds__(kBlock) void k_scatter1(PassArgs a, int32_t rpt, int64_t n_tiles, const uint32_t *rel1,
                                                     const uint64_t *gstart, uint4 *tmp, int total_bits,
                                                     int bin_bits) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    extern __shared__ uint32_t s_cur[];
    const int ng = 1 << (total_bits - bin_bits);
    for (int i = threadIdx.x; i < ng; i += kBlock) s_cur[i] = rel1[(size_t)i * gridDim.x + blockIdx.x];
    fixed_windows<false>(a, rpt, n_tiles, s_b2, s_nm, s_hq, [&](bool act, const Occ &o, int64_t) {
        if (act) {
            const uint32_t g = bin_of(o.hi, o.lo, total_bits) >> bin_bits;
            const uint32_t pos = atomicAdd(&s_cur[g], 1u);
            tmp[gstart[g] + pos] = rec_pack(o);
        }
    });
}

// Level-2 histogram: workgroup (g, slice) counts the bins of its slice of group g's records.
__global__ __launch_bounds__(kBlock) void k_hist2(const uint4 *tmp, const uint64_t *gstart, uint32_t *hist2,
                                                  int total_bits, int bin_bits) {
    extern __shared__ uint32_t s_h[];
    const int ns = 1 << bin_bits;
    const uint32_t g = blockIdx.x / kSlices, sl = blockIdx.x % kSlices;
    for (int i = threadIdx.x; i < ns; i += kBlock) s_h[i] = 0;
    __syncthreads();
    const uint64_t g0 = gstart[g], len = gstart[g + 1] - g0;
    const uint64_t b = g0 + len * sl / kSlices, e = g0 + len * (sl + 1) / kSlices;
    const uint32_t mask = (uint32_t)ns - 1;
    for (uint64_t i0 = b; i0 < e; i0 += kChunk) {
        uint4 r[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = i0 + j * kBlock + threadIdx.x;
            r[j] = i < e ? tmp[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = i0 + j * kBlock + threadIdx.x;
            if (i < e) {
                const Rec x = rec_unpack(r[j]);
                atomicAdd(&s_h[bin_of(x.hi, x.lo, total_bits) & mask], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns; i += kBlock) hist2[((size_t)g * ns + i) * kSlices + sl] = s_h[i];
}

// bin_start[g * ns + s] = group start + offset of (s, slice 0) within the group; the last entry
// closes the final bin.
__global__ __launch_bounds__(kBlock) void k_bin_starts(const uint32_t *rel2, const uint64_t *gstart, uint64_t *bin_start,
                                                       int total_bits, int bin_bits) {
    const uint64_t n_bins = 1ull << total_bits;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i <= n_bins; i += (uint64_t)gridDim.x * kBlock) {
        if (i == n_bins) bin_start[i] = gstart[n_bins >> bin_bits];
        else bin_start[i] = gstart[i >> bin_bits] + rel2[i * kSlices];
    }
}

// Level-2 scatter: workgroup (g, slice) rereads its slice and writes each record to its bin's
// range at the slice's offset.
__global__ __launch_bounds__(kBlock) void k_scatter2(const uint4 *tmp, const uint64_t *gstart, const uint32_t *rel2,
                                                     uint4 *recs, int total_bits, int bin_bits) {
    extern __shared__ uint32_t s_cur[];
    const int ns = 1 << bin_bits;
    const uint32_t g = blockIdx.x / kSlices, sl = blockIdx.x % kSlices;
    for (int i = threadIdx.x; i < ns; i += kBlock) s_cur[i] = rel2[((size_t)g * ns + i) * kSlices + sl];
    __syncthreads();
    const uint64_t g0 = gstart[g], len = gstart[g + 1] - g0;
    const uint64_t b = g0 + len * sl / kSlices, e = g0 + len * (sl + 1) / kSlices;
    const uint32_t mask = (uint32_t)ns - 1;
    for (uint64_t i0 = b; i0 < e; i0 += kChunk) {
        uint4 r[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = i0 + j * kBlock + threadIdx.x;
            r[j] = i < e ? tmp[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = i0 + j * kBlock + threadIdx.x;
            if (i < e) {
                const Rec x = rec_unpack(r[j]);
                const uint32_t pos = atomicAdd(&s_cur[bin_of(x.hi, x.lo, total_bits) & mask], 1u);
                recs[g0 + pos] = r[j];
            }
        }
    }
}

// ------------------------------------------------------------------ counting in LDS

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
};

struct BinLds {
    uint64_t hi[kBinSlots];         // key_hi | kTaken (0 = empty)
    uint64_t lo[kBinSlots];
    uint32_t cnt[9][kBinSlots];     // no left extension, left A..T, right A..T
    uint32_t bloom[kBloomWords];
    uint32_t defer[kDeferCap];      // bin-relative record index of each deferred occurrence
    uint16_t pend[kChunk];          // index within the round of each occurrence to insert
    uint32_t n_pend, n_defer, n_keys, spill;
    unsigned long long base;
};

__device__ __forceinline__ int lds_find(const BinLds &t, uint64_t th, uint64_t lo, uint64_t h) {
    uint32_t s = (uint32_t)h & (kBinSlots - 1);
    for (int p = 0; p < kBinSlots; ++p) {  // the table is never full, so an empty slot ends the probe
        const uint64_t x = t.hi[s];
        if (x == 0) return -1;
        if (x == th && t.lo[s] == lo) return (int)s;
        s = (s + 1) & (kBinSlots - 1);
    }
    return -1;
}

__device__ __forceinline__ void lds_count(BinLds &t, int s, int left, int right) {
    atomicAdd(&t.cnt[left < 4 ? 1 + left : 0][s], 1u);
    if (right < 4) atomicAdd(&t.cnt[5 + right][s], 1u);
}

// Filter word and bits of a key in its bin's Bloom filter (4 bits of one 32-bit word; bits of the
// hash other than those of the home slot).
__device__ __forceinline__ void lds_bloom_bits(uint64_t h, uint32_t &w, uint32_t &m) {
    w = (uint32_t)(h >> 9) & (kBloomWords - 1);
    m = (1u << ((h >> 32) & 31)) | (1u << ((h >> 37) & 31)) | (1u << ((h >> 42) & 31)) | (1u << ((h >> 47) & 31));
}

// Insert (or find) and count the round's pending occurrences: wave 0 alone, while the other
// waves wait at a barrier, so a slot's key words are only written here.  A lane claims an empty
// slot with a compare-and-swap of the first key word and then stores the second; lanes of the
// wave that lost the same slot read both words only after a wave barrier, so they see the
// whole key and either count there (the same key) or probe on.
__device__ __forceinline__ void lds_insert_pending(BinLds &t, const uint4 *R, uint64_t seed, uint32_t &keys_added) {
    // R: the round's first record
    const uint32_t lane = lane_id();
    const uint32_t np = t.n_pend;
    for (uint32_t p0 = 0; p0 < np; p0 += 64) {
        const uint32_t p = p0 + lane;
        bool active = p < np;
        Rec x{0, 0, 4, 4};
        uint32_t s = 0, probes = 0;
        if (active) {
            x = rec_unpack(R[t.pend[p]]);
            s = (uint32_t)key_hash(x.hi, x.lo, seed) & (kBinSlots - 1);
        }
        const uint64_t th = x.hi | kTaken;
        while (__ballot(active)) {
            bool won = false;
            if (active && t.hi[s] == 0) {
                unsigned long long expected = 0;
                won = __hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(&t.hi[s]), &expected,
                                                           (unsigned long long)th, __ATOMIC_RELAXED,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (won) t.lo[s] = x.lo;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (active) {
                if (won) {
                    lds_count(t, (int)s, x.left, x.right);
                    ++keys_added;
                    active = false;
                } else if (t.hi[s] == th && t.lo[s] == x.lo) {
                    lds_count(t, (int)s, x.left, x.right);
                    active = false;
                } else {
                    s = (s + 1) & (kBinSlots - 1);
                    if (++probes >= (uint32_t)kBinSlots) {  // not reached: the key limit keeps a slot free
                        t.spill = 1;
                        active = false;
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_count_bins(CountArgs c, hm_export_t out, hm_occ_t spill) {
    __shared__ BinLds t;
    const uint32_t lane = lane_id();
    const int wave = threadIdx.x >> 6;
    auto clear = [&]() {
        for (int i = threadIdx.x; i < kBinSlots; i += kBlock) t.hi[i] = 0;
        uint4 *cz = reinterpret_cast<uint4 *>(&t.cnt[0][0]);
        for (int i = threadIdx.x; i < 9 * kBinSlots / 4; i += kBlock) cz[i] = make_uint4(0, 0, 0, 0);
        uint4 *bz = reinterpret_cast<uint4 *>(t.bloom);
        for (int i = threadIdx.x; i < kBloomWords / 4; i += kBlock) bz[i] = make_uint4(0, 0, 0, 0);
        if (threadIdx.x == 0) t.n_pend = t.n_defer = t.n_keys = t.spill = 0;
    };
    clear();
    __syncthreads();
    uint64_t dsum = 0, dxor = 0;
    uint64_t st_recs = 0, st_spilled_bins = 0, st_spilled = 0, st_defer = 0, st_keys = 0, st_kept = 0;
    for (uint64_t bin = blockIdx.x; bin < c.n_bins; bin += gridDim.x) {
        const uint64_t b0 = c.bin_start[bin];
        const uint64_t n = c.bin_start[bin + 1] - b0;  // workgroup-uniform
        if (n == 0) continue;
        const uint4 *R = c.recs + b0;
        st_recs += threadIdx.x == 0 ? n : 0;
        // first pass over the bin, a round of kChunk records at a time
        for (uint64_t c0 = 0; c0 < n; c0 += kChunk) {
            uint4 r[kPer];
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const uint64_t i = c0 + j * kBlock + threadIdx.x;
                r[j] = i < n ? R[i] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const uint64_t i = c0 + j * kBlock + threadIdx.x;
                if (i >= n) continue;
                const Rec x = rec_unpack(r[j]);
                const uint64_t h = key_hash(x.hi, x.lo, c.seed);
                const int s = lds_find(t, x.hi | kTaken, x.lo, h);
                if (s >= 0) {
                    lds_count(t, s, x.left, x.right);
                    continue;
                }
                bool seen = c.bypass != 0;
                if (!seen) {
                    uint32_t w, m;
                    lds_bloom_bits(h, w, m);
                    seen = (atomicOr(&t.bloom[w], m) & m) == m;
                }
                if (seen) {
                    t.pend[atomicAdd(&t.n_pend, 1u)] = (uint16_t)(i - c0);
                } else {
                    const uint32_t d = atomicAdd(&t.n_defer, 1u);
                    if (d < (uint32_t)kDeferCap) t.defer[d] = (uint32_t)i;
                    else t.spill = 1;
                }
            }
            __syncthreads();
            if (wave == 0) {
                if (!t.spill) {
                    uint32_t added = 0;
                    lds_insert_pending(t, R + c0, c.seed, added);
                    for (int off = 32; off > 0; off >>= 1) added += __shfl_xor(added, off);
                    if (lane == 0) {
                        t.n_keys += added;
                        if (t.n_keys > kMaxKeys) t.spill = 1;
                    }
                }
                if (lane == 0) t.n_pend = 0;
            }
            __syncthreads();
            if (t.spill) break;
        }
        if (!t.spill) {
            // deferred occurrences: counted when their k-mer is in the table
            const uint32_t nd = t.n_defer;
            for (uint32_t d = threadIdx.x; d < nd; d += kBlock) {
                const Rec x = rec_unpack(R[t.defer[d]]);
                const int s = lds_find(t, x.hi | kTaken, x.lo, key_hash(x.hi, x.lo, c.seed));
                if (s >= 0) lds_count(t, s, x.left, x.right);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                st_defer += nd;
                st_keys += t.n_keys;
            }
            // depth filter, classification and export of the bin's table
            for (int s0 = 0; s0 < kBinSlots; s0 += kBlock) {
                const int s = s0 + threadIdx.x;
                const uint64_t th = t.hi[s];
                bool take = false;
                uint32_t tl[4], tr[4], count = 0, cl = 0, cr = 0;
                if (th) {
                    uint64_t cnt = t.cnt[0][s];
                    for (int q = 0; q < 4; ++q) {
                        tl[q] = t.cnt[1 + q][s];
                        tr[q] = t.cnt[5 + q][s];
                        cnt += tl[q];
                    }
                    count = (uint32_t)cnt;
                    cl = side_class(tl, c.ext_min);
                    cr = side_class(tr, c.ext_min);
                    take = cnt >= c.min_depth && (!c.uu_only || (cl < 4 && cr < 4));
                }
                const uint64_t m = __ballot(take);
                if (m) {
                    const int leader = __ffsll((long long)m) - 1;
                    unsigned long long base = 0;
                    if ((int)lane == leader)
                        base = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_out),
                                         (unsigned long long)__popcll(m));
                    base = __shfl(base, leader);
                    if (take) {
                        const uint64_t idx = base + lanes_below(m);
                        const uint64_t hi = th & ~kTaken, lo = t.lo[s];
                        if (idx < out.capacity) {
                            out.key_hi[idx] = hi;
                            out.key_lo[idx] = lo;
                            out.count[idx] = count;
                            *reinterpret_cast<uint4 *>(out.tl + 4 * idx) = make_uint4(tl[0], tl[1], tl[2], tl[3]);
                            *reinterpret_cast<uint4 *>(out.tr + 4 * idx) = make_uint4(tr[0], tr[1], tr[2], tr[3]);
                            out.cls_l[idx] = (uint8_t)cl;
                            out.cls_r[idx] = (uint8_t)cr;
                        } else {
                            atomicOr(c.status, HM_ST_OUTPUT_FULL);
                        }
                        if (out.digest) {
                            const uint64_t y = record_hash(hi, lo, count, tl, tr, cl, cr);
                            dsum += y;
                            dxor ^= y;
                        }
                        ++st_kept;
                    }
                }
            }
        } else {
            // the bin goes to the global-table path whole
            if (threadIdx.x == 0) {
                t.base = atomicAdd(reinterpret_cast<unsigned long long *>(spill.count), (unsigned long long)n);
                st_spilled_bins += 1;
                st_spilled += n;
            }
            __syncthreads();
            const uint64_t base = t.base;
            for (uint64_t i = threadIdx.x; i < n; i += kBlock) {
                const Rec x = rec_unpack(R[i]);
                const uint64_t idx = base + i;
                if (idx < spill.capacity) {
                    *reinterpret_cast<uint4 *>(spill.keys + 2 * idx) =
                        make_uint4((uint32_t)x.hi, (uint32_t)(x.hi >> 32), (uint32_t)x.lo, (uint32_t)(x.lo >> 32));
                    spill.ext[idx] = (uint8_t)(x.left | (x.right << 4));
                } else {
                    atomicOr(c.status, HM_ST_STREAM_FULL);
                }
            }
        }
        __syncthreads();
        clear();
        __syncthreads();
    }
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

int check_bins(const hm_bins_t *b) {
    if (!b || !b->recs || !b->tmp || !b->scratch || !b->bin_start || !b->status)
        return fail(HM_EINVAL, "bins: a buffer is NULL");
    if (((uintptr_t)b->recs) & 15 || ((uintptr_t)b->tmp) & 15 || ((uintptr_t)b->scratch) & 7)
        return fail(HM_EINVAL, "bins: recs and tmp must be 16-byte aligned, scratch 8-byte aligned");
    if (b->group_bits > (uint32_t)kMaxBits || b->bin_bits > (uint32_t)kMaxBits)
        return fail(HM_EINVAL, "bins: group_bits and bin_bits must be at most %d", kMaxBits);
    return HM_OK;
}

// scratch layout (64-bit words): group starts (ng + 1), group totals (ng), then the two
// histograms (32-bit counters)
struct Scratch {
    uint64_t *gstart, *gtot;
    uint32_t *hist1, *hist2;
};

Scratch scratch_of(const hm_bins_t *b) {
    const uint64_t ng = 1ull << b->group_bits;
    Scratch s;
    s.gstart = b->scratch;
    s.gtot = s.gstart + ng + 1;
    s.hist1 = reinterpret_cast<uint32_t *>(s.gtot + ng);
    s.hist2 = s.hist1 + ng * kGrid1;
    return s;
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

size_t hm_bins_scratch_bytes(uint32_t group_bits, uint32_t bin_bits) {
    if (group_bits > (uint32_t)kMaxBits || bin_bits > (uint32_t)kMaxBits) return 0;
    const uint64_t ng = 1ull << group_bits, nb = 1ull << (group_bits + bin_bits);
    return (size_t)(8 * (2 * ng + 1) + 4 * ng * kGrid1 + 4 * nb * kSlices);
}

int hm_bin_kmers(const hm_reads_t *r, const hm_params_t *p, hm_bins_t *b, hipStream_t s) {
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
    const uint64_t ng = 1ull << b->group_bits, ns = 1ull << b->bin_bits, n_bins = 1ull << total_bits;
    const int64_t W = r->n_reads > 0 ? (int64_t)r->read_len - p->k + 1 : 0;
    const uint64_t windows = W > 0 ? (uint64_t)r->n_reads * (uint64_t)W : 0;
    if (windows > b->capacity) return fail(HM_EINVAL, "bins hold %llu records, the reads have %llu windows",
                                           (unsigned long long)b->capacity, (unsigned long long)windows);
    if (windows >= (1ull << 32)) return fail(HM_EINVAL, "binned counting takes fewer than 2^32 windows per call");
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
    const int32_t rpt = kTileBases / r->read_len;
    const int64_t n_tiles = (r->n_reads + rpt - 1) / rpt;
    const int g1 = (int)(n_tiles < kGrid1 ? n_tiles : kGrid1);
    uint4 *tmp = reinterpret_cast<uint4 *>(b->tmp);
    uint4 *recs = reinterpret_cast<uint4 *>(b->recs);
    hipLaunchKernelGGL(k_hist1, dim3(g1), dim3(kBlock), ng * 4, s, a, rpt, n_tiles, sc.hist1, total_bits, bin_bits);
    hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)ng), dim3(kBlock), 0, s, sc.hist1, g1, sc.gtot);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, s, sc.gtot, (int)ng, sc.gstart);
    hipLaunchKernelGGL(k_scatter1, dim3(g1), dim3(kBlock), ng * 4, s, a, rpt, n_tiles, sc.hist1, sc.gstart, tmp,
                       total_bits, bin_bits);
    const dim3 g2((unsigned)(ng * kSlices));
    hipLaunchKernelGGL(k_hist2, g2, dim3(kBlock), ns * 4, s, tmp, sc.gstart, sc.hist2, total_bits, bin_bits);
    hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)ng), dim3(kBlock), 0, s, sc.hist2, (int)(ns * kSlices),
                       (uint64_t *)nullptr);
    hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)grid_for(n_bins + 1, 16)), dim3(kBlock), 0, s, sc.hist2, sc.gstart,
                       b->bin_start, total_bits, bin_bits);
    hipLaunchKernelGGL(k_scatter2, g2, dim3(kBlock), ns * 4, s, tmp, sc.gstart, sc.hist2, recs, total_bits, bin_bits);
    HM_LAUNCH_CHECK("hm_bin_kmers");
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
    const uint64_t cap = (uint64_t)device_cus() * kCountBlocksPerCu;
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
