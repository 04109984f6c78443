// hm_sort.hip -- key order for exported k-mer records (hm_export_table with
// HM_EXPORT_SORTED).
//
// The records of an export are unordered: compaction writes them in table-slot
// order, which is hash order.  A consumer that merges or binary-searches k-mer
// sets needs them in key order, i.e. lexicographic order of the k-mers (the
// encoding puts the first base in the most significant bits).  Keys travel
// with a 32-bit record index; the rest of each record (count, tallies,
// classes) is written by the export as one 64-byte line per record and
// gathered into place at the end.
//
// Keys of 32 bits or more (k >= 16) are sorted most-significant bits first:
//   1. two stable counting passes on the top 16 key bits (8 bits each, least
//      significant of the two first) group the records by 16-bit prefix, in
//      prefix order;
//   2. k_sort_bounds finds where each of the 65536 prefix groups starts;
//   3. k_sort_groups sorts every group on its own, one workgroup per group:
//      a group of at most 4096 records (about 1500 on average at 10^8
//      records) is ordered in LDS by three counting passes on the next 24 key
//      bits plus an insertion step for the rare ties; a larger group (many
//      distinct k-mers sharing their first 8 bases) takes in-workgroup
//      counting passes through global memory.
// Shorter keys (k < 16, at most 4 digits) take stable counting passes over
// all their digits.  Either way each record crosses memory a few times
// instead of once per 8 key bits.
//
// A counting pass is three kernels:
//   k_sort_hist     one workgroup per 4096-record tile counts the tile's digits
//                   into row `digit` of a digit x tile matrix;
//   k_sort_scan     one workgroup per digit turns its row into exclusive
//                   offsets and stores the row total;
//   k_sort_scatter  each tile ranks its records stably (wave ballots give the
//                   rank among lanes with the same digit; a prefix over item
//                   rounds and waves orders the rest), places them in digit
//                   order in LDS, and writes every digit's run to its global
//                   offset, so consecutive lanes store to consecutive addresses.
// Keys in a table are distinct, so the final order is unique.
#include "hm_device.h"

#include <mutex>

namespace hm {
namespace {

constexpr int kSortIpt = 16;                  // records per thread per tile
constexpr int kSortTile = kBlock * kSortIpt;  // 4096 records
constexpr int kSortWaves = kBlock / 64;
constexpr int kPrefixBits = 16;               // bits of the grouping prefix
constexpr uint32_t kGroups = 1u << kPrefixBits;
constexpr int kGroupMax = 4096;               // records a group sorts in LDS

struct SortLayout {
    uint64_t *hi, *lo;      // key partners of out.key_hi / out.key_lo
    uint32_t *idx0, *idx1;  // record index, ping-pong
    uint4 *pay;             // 4 uint4 per record: tl, tr, {count, cls_l | cls_r << 8}, unused
    uint32_t *hist;         // 256 rows of nblk tile counts
    uint32_t *tot;          // 256 digit totals
    uint32_t *starts;       // kGroups + 1 group starts
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
    L.starts = reinterpret_cast<uint32_t *>(take(4ull * (kGroups + 1)));
    L.bytes = off;
    return L;
}

// Number of records the export produced, clamped to the buffer (on
// HM_ST_OUTPUT_FULL the counter holds the number needed).
__device__ __forceinline__ uint32_t records_in(const uint64_t *n_out, uint64_t cap) {
    const uint64_t n = *n_out;
    return (uint32_t)(n < cap ? n : cap);
}

// Bits [s, s + 64) of the 128-bit key hi:lo, low-aligned.
__device__ __forceinline__ uint64_t key_bits_at(uint64_t hi, uint64_t lo, uint32_t s) {
    if (s >= 64) return hi >> (s - 64);
    return s ? (lo >> s) | (hi << (64 - s)) : lo;
}

__device__ __forceinline__ uint32_t digit_at(uint64_t hi, uint64_t lo, uint32_t s) {
    return (uint32_t)key_bits_at(hi, lo, s) & 255u;
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

// Stable rank of a tile of up to kSortTile records in tile order (item round
// j, then wave, then lane).  dig[j] is the digit of this thread's item j (any
// value when the item is past tile_n).  On return pos[j] is the item's place
// in the tile's digit-sorted order (0xFFFF past tile_n) and tstart[d] the
// first place of digit d, tstart[256] = tile_n.  `cnt` is kSortIpt x waves x
// 256 LDS counters (32 KB), free again on return.  Contains barriers.
__device__ __forceinline__ void tile_rank(const uint32_t (&dig)[kSortIpt], uint32_t tile_n,
                                          uint16_t (*cnt)[kSortWaves][256], uint32_t *tstart, uint32_t *wsum,
                                          uint32_t (&pos)[kSortIpt]) {
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    uint4 *z = reinterpret_cast<uint4 *>(&cnt[0][0][0]);
    for (int i = t; i < kSortIpt * kSortWaves * 256 * 2 / 16; i += kBlock) z[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const uint64_t below_mask = (1ull << lane) - 1;
    uint32_t below[kSortIpt];
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const bool valid = (uint32_t)j * kBlock + t < tile_n;
        const uint32_t d = dig[j] & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        below[j] = (uint32_t)__popcll(m & below_mask);
        if (valid && below[j] == 0) cnt[j][w][d] = (uint16_t)__popcll(m);
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
    if (t == 0) tstart[256] = tile_total;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const bool valid = (uint32_t)j * kBlock + t < tile_n;
        const uint32_t d = dig[j] & 255u;
        pos[j] = valid ? tstart[d] + cnt[j][w][d] + below[j] : 0xFFFFu;
    }
    __syncthreads();
}

// Digit counts of one tile (digit = key bits [shift, shift + 8)); only the
// key words that hold the digit are read.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint64_t *hi, const uint64_t *lo, uint32_t shift,
                                                      const uint64_t *n_out, uint64_t cap, uint32_t *hist,
                                                      uint32_t nblk) {
    __shared__ uint32_t h[kSortWaves][256];
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = records_in(n_out, cap);
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    const int w = threadIdx.x >> 6;
    const bool need_lo = KW == 1 || shift < 64;
    const bool need_hi = KW == 2 && shift + 8 > 64;
    uint32_t d[kSortIpt];
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        const bool ok = i < n;
        const uint64_t l = ok && need_lo ? lo[i] : 0, u = ok && need_hi ? hi[i] : 0;
        d[j] = digit_at(u, l, shift);
    }
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[w][d[j]], 1u);
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

// One stable counting-sort step of a tile on the digit at key bits [shift,
// shift + 8).  KW = key words moved (1 when every key fits key_lo).  FIRST: the
// record index is the input position (no index array yet).
template <int KW, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(const uint64_t *shi, const uint64_t *slo, const uint32_t *sidx,
                                                         uint64_t *dhi, uint64_t *dlo, uint32_t *didx, uint32_t shift,
                                                         const uint64_t *n_out, uint64_t cap, const uint32_t *hist,
                                                         const uint32_t *tot, uint32_t nblk) {
    // the ranking counters and the digit-ordered staging area share 32 KB: the
    // counters are free once every record knows its place in the tile
    __shared__ uint64_t smem[kSortTile];
    __shared__ uint8_t sdig[kSortTile];
    __shared__ uint32_t gbase[256], tstart[257], wsum[kSortWaves];
    static_assert(sizeof(uint16_t) * kSortIpt * kSortWaves * 256 == sizeof(uint64_t) * kSortTile, "LDS overlay");
    uint16_t(*cnt)[kSortWaves][256] = reinterpret_cast<uint16_t(*)[kSortWaves][256]>(smem);

    const uint32_t n = records_in(n_out, cap);
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    if (base >= n) return;  // whole workgroup: past the last record
    const uint32_t tile_n = (uint32_t)min<uint64_t>(kSortTile, n - base);
    const int t = threadIdx.x;

    // global start of digit t for this tile: records of smaller digits, plus
    // digit-t records of earlier tiles
    uint32_t total;
    const uint32_t dstart = block_exclusive(tot[t], wsum, total);
    gbase[t] = dstart + hist[(uint64_t)t * nblk + blockIdx.x];

    uint64_t klo[kSortIpt], khi[KW == 2 ? kSortIpt : 1];
    uint32_t kid[kSortIpt], dig[kSortIpt], pos[kSortIpt];
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        const uint32_t r = (uint32_t)j * kBlock + t;  // tile order: round, then wave, then lane
        const bool valid = r < tile_n;
        const uint64_t i = base + r;
        klo[j] = valid ? slo[i] : 0;
        uint64_t u = 0;
        if constexpr (KW == 2) u = khi[j] = valid ? shi[i] : 0;
        kid[j] = FIRST ? (uint32_t)i : (valid ? sidx[i] : 0u);
        dig[j] = digit_at(u, klo[j], shift);
    }
    tile_rank(dig, tile_n, cnt, tstart, wsum, pos);  // its barriers also publish gbase

#pragma unroll
    for (int j = 0; j < kSortIpt; ++j) {
        if (pos[j] < (uint32_t)kSortTile) {
            sdig[pos[j]] = (uint8_t)dig[j];
            smem[pos[j]] = klo[j];
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
        for (int j = 0; j < kSortIpt; ++j)
            if (pos[j] < (uint32_t)kSortTile) smem[pos[j]] = khi[j];
        __syncthreads();
        for (uint32_t r = t; r < tile_n; r += kBlock) {
            const uint32_t d = sdig[r], g = gbase[d] + (r - tstart[d]);
            if (g < n) dhi[g] = smem[r];
        }
    }
    __syncthreads();
    uint32_t *s32 = reinterpret_cast<uint32_t *>(smem);
#pragma unroll
    for (int j = 0; j < kSortIpt; ++j)
        if (pos[j] < (uint32_t)kSortTile) s32[pos[j]] = kid[j];
    __syncthreads();
    for (uint32_t r = t; r < tile_n; r += kBlock) {
        const uint32_t d = sdig[r], g = gbase[d] + (r - tstart[d]);
        if (g < n) didx[g] = s32[r];
    }
}

// Start of every prefix group in records grouped by their top kPrefixBits key
// bits (bits [pshift, pshift + 16)): starts[P] = first record with prefix >= P,
// starts[kGroups] = n.  Each start is written by the one record where the
// prefix steps past it.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_sort_bounds(const uint64_t *hi, const uint64_t *lo, const uint64_t *n_out,
                                                        uint64_t cap, uint32_t pshift, uint32_t *starts) {
    const uint32_t n = records_in(n_out, cap);
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n == 0) {
        for (uint64_t p = tid; p <= kGroups; p += (uint64_t)gridDim.x * kBlock) starts[p] = 0;
        return;
    }
    for (uint64_t i = tid; i < n; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t p = (uint32_t)key_bits_at(KW == 2 ? hi[i] : 0, lo[i], pshift) & (kGroups - 1);
        const int64_t q = i ? (int64_t)((uint32_t)key_bits_at(KW == 2 ? hi[i - 1] : 0, lo[i - 1], pshift) &
                                        (kGroups - 1))
                            : -1;
        for (int64_t g = q + 1; g <= (int64_t)p; ++g) starts[g] = (uint32_t)i;
        if (i == n - 1)
            for (uint32_t g = p + 1; g <= kGroups; ++g) starts[g] = n;
    }
}

template <int KW>
__device__ __forceinline__ bool key_less(uint64_t ahi, uint64_t alo, uint64_t bhi, uint64_t blo) {
    if constexpr (KW == 2) return ahi < bhi || (ahi == bhi && alo < blo);
    return alo < blo;
}

constexpr int kLowBits = 24;   // key bits below the prefix that the LDS passes sort on
constexpr uint32_t kRunMax = 64;  // longest run of equal top bits ordered by insertion

// Records of a group too large for LDS (or with long runs of equal top bits):
// stable counting passes over all key bits below the prefix, the workgroup
// walking the group tile by tile in order, between the group's ranges of x and
// y; the result ends in y.  `smem` provides the ranking counters and tables.
template <int KW>
__device__ void group_sort_global(uint64_t *xhi, uint64_t *xlo, uint32_t *xid, uint64_t *yhi, uint64_t *ylo,
                                  uint32_t *yid, uint32_t b, uint32_t e, uint32_t pshift, uint64_t *smem) {
    const int t = threadIdx.x;
    uint16_t(*cnt)[kSortWaves][256] = reinterpret_cast<uint16_t(*)[kSortWaves][256]>(smem);
    uint32_t *h = reinterpret_cast<uint32_t *>(smem + kSortTile);  // after the ranking counters
    uint32_t *tstart = h + 256;                                    // 257 entries
    uint32_t *dbase = tstart + 260;                                // 256 entries
    uint32_t *wsum = dbase + 256;                                  // kSortWaves entries
    const int passes = (int)((pshift + 7) / 8);
    // start so that the last pass writes y
    uint64_t *sh_ = xhi, *sl = xlo, *dh = yhi, *dl = ylo;
    uint32_t *si = xid, *di = yid;
    if (!(passes & 1)) {  // an even number of passes: copy to y first, sort y -> x -> ... -> y
        for (uint32_t i = b + t; i < e; i += kBlock) {
            if constexpr (KW == 2) yhi[i] = xhi[i];
            ylo[i] = xlo[i];
            yid[i] = xid[i];
        }
        __syncthreads();
        sh_ = yhi, sl = ylo, dh = xhi, dl = xlo, si = yid, di = xid;
    }
    if (passes == 0) return;  // no bits below the prefix (never for keys of 32 bits or more)
    for (uint32_t shift = 0; shift < pshift; shift += 8) {
        h[t] = 0;
        __syncthreads();
        for (uint32_t i = b + t; i < e; i += kBlock) atomicAdd(&h[digit_at(KW == 2 ? sh_[i] : 0, sl[i], shift)], 1u);
        __syncthreads();
        uint32_t total;
        dbase[t] = b + block_exclusive(h[t], wsum, total);
        __syncthreads();
        for (uint32_t t0 = b; t0 < e; t0 += kSortTile) {
            const uint32_t tile_n = min((uint32_t)kSortTile, e - t0);
            uint32_t dig[kSortIpt], pos[kSortIpt];
#pragma unroll
            for (int j = 0; j < kSortIpt; ++j) {
                const uint32_t r = (uint32_t)j * kBlock + t;
                const bool ok = r < tile_n;
                dig[j] = ok ? digit_at(KW == 2 ? sh_[t0 + r] : 0, sl[t0 + r], shift) : 0u;
            }
            tile_rank(dig, tile_n, cnt, tstart, wsum, pos);
#pragma unroll
            for (int j = 0; j < kSortIpt; ++j) {
                if (pos[j] >= (uint32_t)kSortTile) continue;
                const uint32_t d = dig[j] & 255u;
                const uint32_t g = dbase[d] + (pos[j] - tstart[d]);
                if (g >= e) continue;  // never, when the counts agree
                const uint32_t from = t0 + (uint32_t)j * kBlock + t;  // read again: the tile is cache-resident
                if constexpr (KW == 2) dh[g] = sh_[from];
                dl[g] = sl[from];
                di[g] = si[from];
            }
            __syncthreads();
            dbase[t] += tstart[t + 1] - tstart[t];  // this tile's records of digit t
            __syncthreads();
        }
        uint64_t *x = sh_;
        sh_ = dh;
        dh = x;
        x = sl;
        sl = dl;
        dl = x;
        uint32_t *xi = si;
        si = di;
        di = xi;
    }
}

// Sort every prefix group of x (keys, index) into the same range of y.  One
// workgroup per group.  A group of at most kSortTile records is ordered in LDS
// by permuting 16-bit positions: three stable counting passes on the kLowBits
// key bits below the prefix (the records stay where they are), then runs of
// records whose top bits are all equal, rare for distinct keys, are ordered by
// insertion on the full key; finally the records are gathered from x into y
// in order.  Larger groups, and groups with a run longer than kRunMax, take
// the counting passes through global memory.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_sort_groups(uint64_t *xhi, uint64_t *xlo, uint32_t *xid, uint64_t *yhi,
                                                        uint64_t *ylo, uint32_t *yid, const uint32_t *starts,
                                                        uint32_t pshift, const uint64_t *n_out, uint64_t cap) {
    // 32 KB ranking counters + 16 KB low bits + 2 x 8 KB positions + tables
    constexpr int kWords = kSortTile + kSortTile / 2 + kSortTile / 2 + 320;
    __shared__ uint64_t smem[kWords];
    static_assert(sizeof(uint64_t) * kSortTile + 4 * kSortTile + 2 * 2 * kSortTile + 4 * 264 <= sizeof(uint64_t) * kWords,
                  "group-sort LDS layout");
    static_assert(sizeof(uint64_t) * kSortTile + 4 * 780 <= sizeof(uint64_t) * kWords, "fallback LDS layout");
    __shared__ uint32_t flag;
    const uint32_t n = records_in(n_out, cap);
    const uint32_t b = starts[blockIdx.x], e = min(starts[blockIdx.x + 1], n);  // the clamp only guards the arrays
    if (e <= b) return;
    const uint32_t s = e - b;
    const int t = threadIdx.x;
    if (s > (uint32_t)kSortTile) {
        group_sort_global<KW>(xhi, xlo, xid, yhi, ylo, yid, b, e, pshift, smem);
        return;
    }
    uint16_t(*cnt)[kSortWaves][256] = reinterpret_cast<uint16_t(*)[kSortWaves][256]>(smem);
    uint32_t *low = reinterpret_cast<uint32_t *>(smem + kSortTile);         // kSortTile entries
    uint16_t *perm = reinterpret_cast<uint16_t *>(low + kSortTile);         // 2 x kSortTile entries
    uint32_t *tstart = reinterpret_cast<uint32_t *>(perm + 2 * kSortTile);  // 257 entries
    uint32_t *wsum = tstart + 260;
    const uint32_t lbits = pshift < (uint32_t)kLowBits ? pshift : (uint32_t)kLowBits;
    const uint32_t lshift = pshift - lbits;
    const uint32_t lmask = (1u << lbits) - 1;
    if (t == 0) flag = 0;
    for (uint32_t q = t; q < s; q += kBlock) {
        low[q] = (uint32_t)key_bits_at(KW == 2 ? xhi[b + q] : 0, xlo[b + q], lshift) & lmask;
        perm[q] = (uint16_t)q;
    }
    __syncthreads();
    uint16_t *cur = perm, *nxt = perm + kSortTile;
    for (uint32_t shift = 0; shift < lbits; shift += 8) {
        uint32_t dig[kSortIpt], pos[kSortIpt], src[kSortIpt];
#pragma unroll
        for (int j = 0; j < kSortIpt; ++j) {
            const uint32_t q = (uint32_t)j * kBlock + t;
            src[j] = q < s ? cur[q] : 0u;
            dig[j] = (low[src[j]] >> shift) & 255u;
        }
        tile_rank(dig, s, cnt, tstart, wsum, pos);
#pragma unroll
        for (int j = 0; j < kSortIpt; ++j)
            if (pos[j] < s) nxt[pos[j]] = (uint16_t)src[j];
        __syncthreads();
        uint16_t *x = cur;
        cur = nxt;
        nxt = x;
    }
    // runs of equal low bits: order them by the full key (they share all the top bits)
    if (lshift > 0) {
        for (uint32_t q = t; q + 1 < s; q += kBlock) {
            const uint32_t v = low[cur[q]];
            if ((q > 0 && low[cur[q - 1]] == v) || low[cur[q + 1]] != v) continue;  // not the start of a run
            uint32_t r = q + 1;
            while (r < s && low[cur[r]] == v) ++r;
            if (r - q > kRunMax) {
                atomicOr(&flag, 1u);
                continue;
            }
            for (uint32_t i = q + 1; i < r; ++i) {  // insertion sort of cur[q..r) by key
                const uint16_t pi = cur[i];
                const uint64_t ih = KW == 2 ? xhi[b + pi] : 0, il = xlo[b + pi];
                uint32_t j = i;
                while (j > q) {
                    const uint16_t pj = cur[j - 1];
                    if (!key_less<KW>(ih, il, KW == 2 ? xhi[b + pj] : 0, xlo[b + pj])) break;
                    cur[j] = pj;
                    --j;
                }
                cur[j] = pi;
            }
        }
        __syncthreads();
        if (flag) {  // a long run of equal top bits: take the general path
            group_sort_global<KW>(xhi, xlo, xid, yhi, ylo, yid, b, e, pshift, smem);
            return;
        }
    }
    for (uint32_t q = t; q < s; q += kBlock) {
        const uint32_t from = b + cur[q];
        if constexpr (KW == 2) yhi[b + q] = xhi[from];
        ylo[b + q] = xlo[from];
        yid[b + q] = xid[from];
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

// One stable counting pass (hist, scan, scatter) from (shi, slo, sidx) to
// (dhi, dlo, didx) on key bits [shift, shift + 8); sidx NULL: first pass.
template <int KW>
int counting_pass(const hm_export_t &out, const SortLayout &L, const uint64_t *shi, const uint64_t *slo,
                  const uint32_t *sidx, uint64_t *dhi, uint64_t *dlo, uint32_t *didx, uint32_t shift, hipStream_t s) {
    const dim3 tiles(L.nblk), blk(kBlock);
    hipLaunchKernelGGL(k_sort_hist<KW>, tiles, blk, 0, s, shi, slo, shift, out.n_out, out.capacity, L.hist, L.nblk);
    hipLaunchKernelGGL(k_sort_scan, dim3(256), blk, 0, s, L.hist, L.nblk, L.tot);
    if (!sidx)
        hipLaunchKernelGGL((k_sort_scatter<KW, true>), tiles, blk, 0, s, shi, slo, nullptr, dhi, dlo, didx, shift,
                           out.n_out, out.capacity, L.hist, L.tot, L.nblk);
    else
        hipLaunchKernelGGL((k_sort_scatter<KW, false>), tiles, blk, 0, s, shi, slo, sidx, dhi, dlo, didx, shift,
                           out.n_out, out.capacity, L.hist, L.tot, L.nblk);
    HM_LAUNCH_CHECK("sort pass");
    return HM_OK;
}

template <int KW>
int sort_keys(const hm_export_t &out, const SortLayout &L, int key_bits, hipStream_t s) {
    const dim3 blk(kBlock);
    uint64_t *kh[2] = {out.key_hi, L.hi};
    uint64_t *kl[2] = {out.key_lo, L.lo};
    uint32_t *ix[2] = {L.idx0, L.idx1};
    const dim3 sweep((unsigned)grid_for(out.capacity, 16));
    int rc;
    if (key_bits < 2 * kPrefixBits) {  // short keys: a counting pass per digit
        const int passes = (key_bits + 7) / 8;
        for (int p = 0; p < passes; ++p) {
            const int src = p & 1, dst = src ^ 1;
            rc = counting_pass<KW>(out, L, kh[src], kl[src], p ? ix[(p - 1) & 1] : nullptr, kh[dst], kl[dst],
                                   ix[p & 1], 8u * (uint32_t)p, s);
            if (rc) return rc;
        }
        const int res = passes & 1;  // 1: the sorted keys are in the work area
        hipLaunchKernelGGL(k_sort_final<KW>, sweep, blk, 0, s, kh[res], kl[res], ix[(passes - 1) & 1], L.pay, out, res);
        HM_LAUNCH_CHECK("sort gather");
        return HM_OK;
    }
    // group by the top 16 bits (two passes, the lower byte first), then sort each group
    const uint32_t pshift = (uint32_t)key_bits - kPrefixBits;
    rc = counting_pass<KW>(out, L, kh[0], kl[0], nullptr, kh[1], kl[1], ix[0], pshift, s);
    if (rc) return rc;
    rc = counting_pass<KW>(out, L, kh[1], kl[1], ix[0], kh[0], kl[0], ix[1], pshift + 8, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sort_bounds<KW>, sweep, blk, 0, s, kh[0], kl[0], out.n_out, out.capacity, pshift, L.starts);
    hipLaunchKernelGGL(k_sort_groups<KW>, dim3(kGroups), blk, 0, s, kh[0], kl[0], ix[1], kh[1], kl[1], ix[0],
                       L.starts, pshift, out.n_out, out.capacity);
    HM_LAUNCH_CHECK("sort groups");
    hipLaunchKernelGGL(k_sort_final<KW>, sweep, blk, 0, s, kh[1], kl[1], ix[0], L.pay, out, 1);
    HM_LAUNCH_CHECK("sort gather");
    return HM_OK;
}

}  // namespace

uint64_t sort_work_bytes(uint64_t capacity) { return sort_layout(nullptr, capacity).bytes; }

uint4 *sort_staging(const hm_export_t &out) { return sort_layout(out.sort_work, out.capacity).pay; }

// The export has written keys to out.key_* and the rest of every record to
// sort_staging(out).
int sort_export(const hm_export_t &out, int key_bits, hipStream_t s) {
    if (out.capacity == 0) return HM_OK;
    const SortLayout L = sort_layout(out.sort_work, out.capacity);
    return key_bits > 64 ? sort_keys<2>(out, L, key_bits, s) : sort_keys<1>(out, L, key_bits, s);
}

// ------------------------------------------------------------------ scratch held by the library

// The key-ordered export's scratch for callers that cannot allocate
// (hm_export_table_static): a device array of the library's code object,
// allocated on each GPU when the library is loaded there and held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name is only a stand-in): the array's device address is looked up
// once per device and kept in g_scratch.
constexpr uint64_t kStaticRecords = HM_EXPORT_STATIC_MAX_RECORDS;
constexpr uint64_t kStaticBytes = 24ull << 20;  // >= sort_work_bytes(kStaticRecords), checked at first use

static __device__ __align__(256) uint8_t scratch[kStaticBytes];

static std::mutex g_scratch_mu;
static void *g_scratch[64];

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
static int static_scratch(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(HM_EINVAL, "device %d out of range for the static scratch", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (((uintptr_t)p) & 255)) return fail(HM_EHIP, "static scratch: bad device address %p", p);
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return HM_OK;
}

}  // namespace hm

extern "C" size_t hm_export_sort_bytes(uint64_t capacity) { return (size_t)hm::sort_work_bytes(capacity); }

extern "C" int hm_export_table_static(const hm_table_t *t, uint32_t flags, hm_export_t *out, hipStream_t s) {
    using namespace hm;
    if (!(flags & HM_EXPORT_SORTED)) return hm_export_table(t, flags, out, s);  // no scratch needed
    if (!out) return fail(HM_EINVAL, "export: out is NULL");
    if (out->capacity > kStaticRecords)
        return fail(HM_EINVAL, "hm_export_table_static: export capacity %llu exceeds the static scratch's %llu records",
                    (unsigned long long)out->capacity, (unsigned long long)kStaticRecords);
    static_assert(kStaticRecords < (1ull << 32), "record indices are 32-bit");
    if (sort_work_bytes(kStaticRecords) > kStaticBytes)
        return fail(HM_EINVAL, "static scratch of %llu bytes is smaller than the %llu a sort of %llu records needs",
                    (unsigned long long)kStaticBytes, (unsigned long long)sort_work_bytes(kStaticRecords),
                    (unsigned long long)kStaticRecords);
    void *p = nullptr;
    const int rc = static_scratch(&p);
    if (rc) return rc;
    hm_export_t o = *out;  // the same outputs; only the scratch differs
    o.sort_work = p;
    o.sort_work_bytes = kStaticBytes;
    return hm_export_table(t, flags, &o, s);
}
