// hm_sort.hip -- key order for exported k-mer records (hm_export_table with
// HM_EXPORT_SORTED).
//
// The records of an export are unordered: compaction writes them in table-slot
// order, which is hash order.  A consumer that merges or binary-searches k-mer
// sets needs them in key order, i.e. lexicographic order of the k-mers (the
// encoding puts the first base in the most significant bits).  The sort is a
// least-significant-digit radix sort over the 2k key bits, 8 bits per pass.
// Keys travel with a 32-bit record index; the rest of each record (count,
// tallies, classes) is staged once as one 64-byte line per record and gathered
// into place after the last pass, so a pass moves 20 bytes per record (12 for
// k <= 32, whose keys fit one word) instead of 54.
//
// Each pass is three kernels:
//   k_sort_hist     one workgroup per 4096-record tile counts the tile's digits
//                   into row `digit` of a digit x tile matrix;
//   k_sort_scan     one workgroup per digit turns its row into exclusive
//                   offsets and stores the row total;
//   k_sort_scatter  each tile ranks its records stably (wave ballots give the
//                   rank among lanes with the same digit; a prefix over item
//                   rounds and waves orders the rest), places them in digit
//                   order in LDS, and writes every digit's run to its global
//                   offset, so consecutive lanes store to consecutive addresses.
// Stability of every pass is what makes the LSD order correct; keys in a
// table are distinct, so the final order is unique.
#include "hm_device.h"

namespace hm {
namespace {

constexpr int kSortIpt = 16;                  // records per thread per tile
constexpr int kSortTile = kBlock * kSortIpt;  // 4096 records
constexpr int kSortWaves = kBlock / 64;

struct SortLayout {
    uint64_t *hi, *lo;      // key partners of out.key_hi / out.key_lo
    uint32_t *idx0, *idx1;  // record index, ping-pong
    uint4 *pay;             // 4 uint4 per record: tl, tr, {count, cls_l | cls_r << 8}, unused
    uint32_t *hist;         // 256 rows of nblk tile counts
    uint32_t *tot;          // 256 digit totals
    uint32_t nblk;
    uint64_t bytes;
};

inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

SortLayout sort_layout(void *work, uint64_t cap) {
    SortLayout L{};
    const uint64_t nblk = cap ? (cap + kSortTile - 1) / kSortTile : 1;
    L.nblk = (uint32_t)nblk;
    uint64_t off = 0;
    auto take = [&](uint64_t n) {
        const uint64_t o = off;
        off = align256(off + n);
        return reinterpret_cast<char *>(work) + o;
    };
    L.hi = reinterpret_cast<uint64_t *>(take(8 * cap));
    L.lo = reinterpret_cast<uint64_t *>(take(8 * cap));
    L.idx0 = reinterpret_cast<uint32_t *>(take(4 * cap));
    L.idx1 = reinterpret_cast<uint32_t *>(take(4 * cap));
    L.pay = reinterpret_cast<uint4 *>(take(64 * cap));
    L.hist = reinterpret_cast<uint32_t *>(take(4ull * 256 * nblk));
    L.tot = reinterpret_cast<uint32_t *>(take(4ull * 256));
    L.bytes = off;
    return L;
}

// Number of records the export produced, clamped to the buffer (on
// HM_ST_OUTPUT_FULL the counter holds the number needed).
__device__ __forceinline__ uint32_t records_in(const uint64_t *n_out, uint64_t cap) {
    const uint64_t n = *n_out;
    return (uint32_t)(n < cap ? n : cap);
}

// Exclusive prefix sum over the kBlock threads of a workgroup; every thread
// gets the workgroup total.  Contains barriers: call from all threads.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < kSortWaves; ++i) {
        const uint32_t s = wsum[i];
        before += i < w ? s : 0u;
        total += s;
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_sort_prep(hm_export_t out, uint4 *pay) {
    const uint32_t n = records_in(out.n_out, out.capacity);
    const uint4 *tl = reinterpret_cast<const uint4 *>(out.tl);
    const uint4 *tr = reinterpret_cast<const uint4 *>(out.tr);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
        pay[4 * i] = tl[i];
        pay[4 * i + 1] = tr[i];
        pay[4 * i + 2] = make_uint4(out.count[i], out.cls_l[i] | (uint32_t)out.cls_r[i] << 8, 0u, 0u);
    }
}

// Digit counts of one tile: `word` is the key word holding the digit, `shift`
// its position in that word.
__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint64_t *word, uint32_t shift, const uint64_t *n_out,
                                                      uint64_t cap, uint32_t *hist, uint32_t nblk) {
    __shared__ uint32_t h[kSortWaves][256];
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = records_in(n_out, cap);
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    const int w = threadIdx.x >> 6;
    uint64_t v[kSortIpt];
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        v[j] = i < n ? word[i] : 0;
    }
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[w][(v[j] >> shift) & 255], 1u);
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) s += h[q][threadIdx.x];
    hist[(uint64_t)threadIdx.x * nblk + blockIdx.x] = s;
}

// Row `blockIdx.x` (one digit) of the tile-count matrix -> exclusive offsets
// within that digit; tot[digit] = the digit's total.
__global__ __launch_bounds__(kBlock) void k_sort_scan(uint32_t *hist, uint32_t nblk, uint32_t *tot) {
    __shared__ uint32_t wsum[kSortWaves];
    uint32_t *row = hist + (uint64_t)blockIdx.x * nblk;
    const uint32_t seg = (nblk + kBlock - 1) / kBlock;
    const uint32_t b0 = min(nblk, threadIdx.x * seg), b1 = min(nblk, b0 + seg);
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += row[b];
    uint32_t total;
    uint32_t run = block_exclusive(s, wsum, total);
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t v = row[b];
        row[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// One stable counting-sort step of a tile on the digit at bit `shift` of the
// 128-bit key (hi:lo).  KW = key words moved (1 when every key fits key_lo).
// FIRST: the record index is the input position (no index array yet).
template <int KW, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(const uint64_t *shi, const uint64_t *slo, const uint32_t *sidx,
                                                         uint64_t *dhi, uint64_t *dlo, uint32_t *didx, uint32_t shift,
                                                         const uint64_t *n_out, uint64_t cap, const uint32_t *hist,
                                                         const uint32_t *tot, uint32_t nblk) {
    // cnt[j][w][d] (records of digit d among item round j of wave w) and the
    // digit-ordered staging area share the same 32 KB: the counts are dead
    // once every record knows its tile position.
    __shared__ uint64_t smem[kSortTile];
    __shared__ uint8_t sdig[kSortTile];
    __shared__ uint32_t gbase[256], tstart[256], wsum[kSortWaves];
    static_assert(sizeof(uint16_t) * kSortIpt * kSortWaves * 256 == sizeof(uint64_t) * kSortTile, "LDS overlay");
    uint16_t(*cnt)[kSortWaves][256] = reinterpret_cast<uint16_t(*)[kSortWaves][256]>(smem);

    const uint32_t n = records_in(n_out, cap);
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    if (base >= n) return;  // whole workgroup: past the last record
    const uint32_t tile_n = (uint32_t)min<uint64_t>(kSortTile, n - base);
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;

    uint4 *z = reinterpret_cast<uint4 *>(smem);
    for (int i = t; i < kSortTile * 8 / 16; i += kBlock) z[i] = make_uint4(0u, 0u, 0u, 0u);
    // global start of digit t for this tile: records of smaller digits, plus
    // digit-t records of earlier tiles (block_exclusive's barrier also orders
    // the zeroing above before the counts below)
    uint32_t total;
    const uint32_t dstart = block_exclusive(tot[t], wsum, total);
    gbase[t] = dstart + hist[(uint64_t)t * nblk + blockIdx.x];

    const bool dig_hi = shift >= 64;
    const uint32_t sh = shift & 63;
    const uint64_t below_mask = (1ull << lane) - 1;
    uint64_t klo[kSortIpt], khi[KW == 2 ? kSortIpt : 1];
    uint32_t kid[kSortIpt], meta[kSortIpt];
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint32_t r = (uint32_t)j * kBlock + t;  // tile order: round, then wave, then lane
        const bool valid = r < tile_n;
        const uint64_t i = base + r;
        klo[j] = valid ? slo[i] : 0;
        if constexpr (KW == 2) khi[j] = valid ? shi[i] : 0;
        kid[j] = FIRST ? (uint32_t)i : (valid ? sidx[i] : 0u);
    }
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const bool valid = (uint32_t)j * kBlock + t < tile_n;
        uint64_t dw = klo[j];
        if constexpr (KW == 2) dw = dig_hi ? khi[j] : dw;
        const uint32_t d = (uint32_t)(dw >> sh) & 255;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(m & below_mask);
        if (valid && below == 0) cnt[j][w][d] = (uint16_t)__popcll(m);
        meta[j] = d | below << 8;
    }
    __syncthreads();
    // thread t owns digit t: running count over (round, wave) in tile order
    uint32_t run = 0;
    for (int j = 0; j < kSortIpt; ++j)
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) {
            const uint32_t c = cnt[j][q][t];
            cnt[j][q][t] = (uint16_t)run;
            run += c;
        }
    uint32_t tile_total;
    tstart[t] = block_exclusive(run, wsum, tile_total);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const bool valid = (uint32_t)j * kBlock + t < tile_n;
        const uint32_t d = meta[j] & 255;
        const uint32_t pos = valid ? tstart[d] + cnt[j][w][d] + (meta[j] >> 8) : 0xFFFFu;
        meta[j] = d | pos << 8;
    }
    __syncthreads();  // counts dead from here on: smem becomes the staging area

#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint32_t pos = meta[j] >> 8;
        if (pos < (uint32_t)kSortTile) {
            sdig[pos] = (uint8_t)(meta[j] & 255);
            smem[pos] = klo[j];
        }
    }
    __syncthreads();
    // every destination is below n when the counts agree; the guard keeps a
    // disagreement from writing outside the arrays
    for (uint32_t r = t; r < tile_n; r += kBlock) {
        const uint32_t d = sdig[r], g = gbase[d] + (r - tstart[d]);
        if (g < n) dlo[g] = smem[r];
    }
    if constexpr (KW == 2) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortIpt; ++j) {
            const uint32_t pos = meta[j] >> 8;
            if (pos < (uint32_t)kSortTile) smem[pos] = khi[j];
        }
        __syncthreads();
        for (uint32_t r = t; r < tile_n; r += kBlock) {
            const uint32_t d = sdig[r], g = gbase[d] + (r - tstart[d]);
            if (g < n) dhi[g] = smem[r];
        }
    }
    __syncthreads();
    uint32_t *s32 = reinterpret_cast<uint32_t *>(smem);
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint32_t pos = meta[j] >> 8;
        if (pos < (uint32_t)kSortTile) s32[pos] = kid[j];
    }
    __syncthreads();
    for (uint32_t r = t; r < tile_n; r += kBlock) {
        const uint32_t d = sdig[r], g = gbase[d] + (r - tstart[d]);
        if (g < n) didx[g] = s32[r];
    }
}

// Gather count, tallies and classes into key order; copy the sorted keys into
// the export when the last pass left them in the work area.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_sort_final(const uint64_t *khi, const uint64_t *klo, const uint32_t *idx,
                                                       const uint4 *pay, hm_export_t out, int copy_keys) {
    const uint32_t n = records_in(out.n_out, out.capacity);
    uint4 *tl = reinterpret_cast<uint4 *>(out.tl);
    uint4 *tr = reinterpret_cast<uint4 *>(out.tr);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t ji = idx[i];
        const uint64_t j = ji < n ? ji : i;  // an index is always < n; never read past the staged records
        const uint4 a = pay[4 * j], b = pay[4 * j + 1], c = pay[4 * j + 2];
        tl[i] = a;
        tr[i] = b;
        out.count[i] = c.x;
        out.cls_l[i] = (uint8_t)(c.y & 255);
        out.cls_r[i] = (uint8_t)(c.y >> 8);
        if (copy_keys) {
            out.key_lo[i] = klo[i];
            if constexpr (KW == 2) out.key_hi[i] = khi[i];
        }
    }
}

template <int KW>
int sort_passes(const hm_export_t &out, const SortLayout &L, int passes, hipStream_t s) {
    const dim3 tiles(L.nblk), blk(kBlock);
    uint64_t *kh[2] = {out.key_hi, L.hi};
    uint64_t *kl[2] = {out.key_lo, L.lo};
    uint32_t *ix[2] = {L.idx0, L.idx1};
    for (int p = 0; p < passes; ++p) {
        const uint32_t shift = 8u * (uint32_t)p;
        const int src = p & 1, dst = src ^ 1;
        const uint64_t *word = shift >= 64 ? kh[src] : kl[src];
        hipLaunchKernelGGL(k_sort_hist, tiles, blk, 0, s, word, shift & 63u, out.n_out, out.capacity, L.hist, L.nblk);
        hipLaunchKernelGGL(k_sort_scan, dim3(256), blk, 0, s, L.hist, L.nblk, L.tot);
        if (p == 0)
            hipLaunchKernelGGL((k_sort_scatter<KW, true>), tiles, blk, 0, s, kh[src], kl[src], nullptr, kh[dst],
                               kl[dst], ix[0], shift, out.n_out, out.capacity, L.hist, L.tot, L.nblk);
        else
            hipLaunchKernelGGL((k_sort_scatter<KW, false>), tiles, blk, 0, s, kh[src], kl[src], ix[(p - 1) & 1],
                               kh[dst], kl[dst], ix[p & 1], shift, out.n_out, out.capacity, L.hist, L.tot, L.nblk);
        HM_LAUNCH_CHECK("sort pass");
    }
    const int res = passes & 1;  // 1: the sorted keys are in the work area
    hipLaunchKernelGGL(k_sort_final<KW>, dim3((unsigned)grid_for(out.capacity, 16)), blk, 0, s, kh[res], kl[res],
                       ix[(passes - 1) & 1], L.pay, out, res);
    HM_LAUNCH_CHECK("sort gather");
    return HM_OK;
}

}  // namespace

uint64_t sort_work_bytes(uint64_t capacity) { return sort_layout(nullptr, capacity).bytes; }

int sort_export(const hm_export_t &out, int key_bits, hipStream_t s) {
    if (out.capacity == 0) return HM_OK;
    const SortLayout L = sort_layout(out.sort_work, out.capacity);
    hipLaunchKernelGGL(k_sort_prep, dim3((unsigned)grid_for(out.capacity, 16)), dim3(kBlock), 0, s, out, L.pay);
    HM_LAUNCH_CHECK("sort prep");
    const int passes = (key_bits + 7) / 8;
    return key_bits > 64 ? sort_passes<2>(out, L, passes, s) : sort_passes<1>(out, L, passes, s);
}

}  // namespace hm

extern "C" size_t hm_export_sort_bytes(uint64_t capacity) { return (size_t)hm::sort_work_bytes(capacity); }
