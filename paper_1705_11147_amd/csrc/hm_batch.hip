// Batched form of k-mer analysis: many read sets in one persistent launch.
//
// Same method and per-occurrence code as the plain path (hm_kmer.hip, arXiv
// 1705.11147 section "Parallel k-mer analysis"); what changes is scheduling.
// A batch of read sets of uneven size runs as three graph-capturable launches:
//   1. k_fill_regions clears every set's table, filter, counters;
//   2. k_pack_batch packs every set's reads;
//   3. k_batch, a persistent kernel.  Its blocks take work items from one
//      atomic ticket.  Items of a set are its pass-1 runs of reads (staged in
//      LDS one tile at a time) followed by its pass-2 first-occurrence list
//      ranges; sets run larger first, either one after another (set-major:
//      only one or two sets' tables are live at a time, so they stay in the
//      memory-side cache) or phase by phase.  A pass-2 item of set s waits
//      until every pass-1 item of s has finished: per-set counters, one
//      release atomic add per finished item (thread 0, after the workgroup
//      barrier), one acquire by the waiting block's thread 0 (an agent-scope
//      release or acquire is an L2 write-back or invalidate of the XCD on
//      this GPU, so each is made once per item, not once per wave).  A waiter only
//      ever waits on items with smaller tickets, which running blocks already
//      hold, so the schedule cannot deadlock; the wait is still bounded in
//      time and reports HM_ST_TIMEOUT instead of hanging;
//   4. k_export_batch classifies and exports every set (its own launch, so
//      the counting kernel keeps the register budget of pass 1).
// Small sets therefore share the machine instead of each paying a full
// sequence of under-filled launches, and one set's pass 2 overlaps another
// set's pass 1.
#include <stddef.h>

#include <algorithm>
#include <vector>

#include "hm_device.h"

namespace {

using namespace hm;

constexpr int kPhases = 2;  // persistent kernel: pass 1, pass 2
constexpr uint64_t kWaitTicks = 100ull * 1000 * 1000 * 20;  // 20 s at the 100 MHz wall clock

struct BatchDesc {
    const uint8_t *ascii, *qual;
    uint64_t *b2, *nm, *hq;
    int64_t n_reads, n_bases;
    uint64_t n_mask_words;
    int32_t read_len, rpt;  // reads per pass-1 item
    Slot *slots;
    uint64_t capacity;
    uint32_t max_probe;
    uint32_t *status;
    unsigned long long *stats;
    uint64_t *bloom;
    uint64_t bloom_mask;
    uint32_t n_hash;
    uint64_t *lkeys;
    uint8_t *lext;
    uint64_t lcap;
    unsigned long long *lcount;
    uint64_t *present;
    uint64_t present_words;
    uint32_t present_hash;
    hm_export_t out;
    int64_t n_items[kPhases];
    int64_t n_export_items;
};

struct Region {
    void *p;           // any alignment
    uint64_t bytes;    // any count
    uint32_t pattern;  // fill byte, replicated into all four bytes (0 or 0xFFFFFFFF here)
    uint32_t pad;
};

struct BatchHeader {
    int32_t n_sets;
    int32_t k;
    uint32_t forward_only, n_owners, owner, bypass, min_depth, ext_min, export_flags, checked;
    int32_t qual_offset, qcut;
    int32_t list_per_item, slots_per_item;
    int64_t n_items;
    uint64_t seed;
    // cleared at every launch:
    unsigned long long ticket;
    uint32_t pad[2];
};

// work blob layout: header | descs[S] | item_start[2S+1] | group[2S] | pack_start[S+1] | export_start[S+1] |
// regions[R] | done[2S].  Ticket group g covers items [item_start[g], item_start[g+1]) of phase
// group[g] >> 24 of set group[g] & 0xFFFFFF.
struct Layout {
    size_t desc, item_start, group, pack_start, export_start, regions, done, total;
};

constexpr int kRegionsPerSet = 9;

Layout layout(int32_t S) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    Layout l;
    l.desc = up(sizeof(BatchHeader));
    l.item_start = up(l.desc + sizeof(BatchDesc) * S);
    l.group = up(l.item_start + sizeof(int64_t) * (kPhases * S + 1));
    l.pack_start = up(l.group + sizeof(int32_t) * kPhases * S);
    l.export_start = up(l.pack_start + sizeof(int64_t) * (S + 1));
    l.regions = up(l.export_start + sizeof(int64_t) * (S + 1));
    l.done = up(l.regions + sizeof(Region) * (kRegionsPerSet * S + 1));
    l.total = up(l.done + sizeof(uint32_t) * kPhases * S);
    return l;
}

// ------------------------------------------------------------------ kernels

// Fill exactly r.bytes bytes of region blockIdx.y with its pattern byte:
// single bytes up to the first 16-byte boundary and after the last one,
// 16-byte stores between them.
__global__ __launch_bounds__(kBlock) void k_fill_regions(const Region *regions) {
    const Region r = regions[blockIdx.y];
    if (!r.p || r.bytes == 0) return;
    uint8_t *p = reinterpret_cast<uint8_t *>(r.p);
    const uint32_t v = r.pattern;
    const uint8_t byte = (uint8_t)v;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t head = (16 - (((uintptr_t)p) & 15)) & 15;
    if (head > r.bytes) head = r.bytes;
    const uint64_t n16 = (r.bytes - head) / 16;
    for (uint64_t i = tid; i < head; i += stride) p[i] = byte;
    uint4 *q = reinterpret_cast<uint4 *>(p + head);
    for (uint64_t i = tid; i < n16; i += stride) q[i] = make_uint4(v, v, v, v);
    for (uint64_t i = head + 16 * n16 + tid; i < r.bytes; i += stride) p[i] = byte;
}

__device__ __forceinline__ int find_range(const int64_t *start, int n, int64_t t) {
    int lo = 0, hi = n;  // last i with start[i] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Pack every set's reads; one thread per mask word over the concatenation.
__global__ __launch_bounds__(kBlock) void k_pack_batch(const BatchHeader *hdr, const BatchDesc *sets,
                                                       const int64_t *pack_start) {
    const int S = hdr->n_sets;
    const int64_t total = pack_start[S];
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < total; g += (int64_t)gridDim.x * kBlock) {
        const int s = find_range(pack_start, S, g);
        const BatchDesc &d = sets[s];
        const uint64_t m = (uint64_t)(g - pack_start[s]);
        const int64_t base = (int64_t)m * 64;
        uint64_t c0 = 0, c1 = 0, nmask = ~0ull, hmask = 0;
        if (base < d.n_bases) {
            const int cnt = (int)min((int64_t)64, d.n_bases - base);
            const bool aligned = ((((uintptr_t)d.ascii) | ((uintptr_t)d.qual)) & 15) == 0;
            nmask = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nv = cnt - 16 * v;
                uint4 sa = make_uint4(0, 0, 0, 0), sq = make_uint4(0, 0, 0, 0);
                if (nv >= 16 && aligned) {
                    sa = *reinterpret_cast<const uint4 *>(d.ascii + base + 16 * v);
                    sq = *reinterpret_cast<const uint4 *>(d.qual + base + 16 * v);
                } else if (nv > 0) {
                    uint32_t ta[4] = {0, 0, 0, 0}, tq[4] = {0, 0, 0, 0};
                    for (int i = 0; i < 16 && i < nv; ++i) {
                        ta[i >> 2] |= (uint32_t)d.ascii[base + 16 * v + i] << (8 * (i & 3));
                        tq[i >> 2] |= (uint32_t)d.qual[base + 16 * v + i] << (8 * (i & 3));
                    }
                    sa = make_uint4(ta[0], ta[1], ta[2], ta[3]);
                    sq = make_uint4(tq[0], tq[1], tq[2], tq[3]);
                }
                uint64_t codes;
                uint32_t bad, good;
                pack16(sa, sq, nv, hdr->qual_offset, hdr->qcut, codes, bad, good);
                if (v < 2) c0 |= codes << (32 * (1 - v));
                else c1 |= codes << (32 * (3 - v));
                nmask |= (uint64_t)bad << (16 * (3 - v));
                hmask |= (uint64_t)good << (16 * (3 - v));
            }
        }
        d.b2[2 * m] = c0;
        d.b2[2 * m + 1] = c1;
        d.nm[m] = nmask;
        d.hq[m] = hmask;
    }
}

// A set's descriptor is written by the host before the launch and never by a
// kernel, so it is read through the constant address space: the compiler may
// then load its fields again where needed instead of holding them in
// registers (the persistent kernel fits eight waves per SIMD without spills).
typedef const __attribute__((address_space(4))) BatchDesc ConstDesc;

__device__ __forceinline__ PassArgs pass_args(const BatchHeader *hdr, const BatchDesc &dg) {
    const ConstDesc &d = *(ConstDesc *)&dg;
    PassArgs a;
    a.b2 = d.b2;
    a.nm = d.nm;
    a.hq = d.hq;
    a.read_off = nullptr;
    a.n_reads = d.n_reads;
    a.n_bases = d.n_bases;
    a.read_len = d.read_len;
    a.k = hdr->k;
    a.forward_only = hdr->forward_only;
    a.n_owners = hdr->n_owners;
    a.owner = hdr->owner;
    a.seed = hdr->seed;
    a.bloom = d.bloom;
    a.bloom_mask = d.bloom_mask;
    a.n_hash = d.n_hash;
    a.bypass = hdr->bypass;
    a.slots = d.slots;
    a.cmask = d.capacity - 1;
    a.max_probe = d.max_probe;
    a.status = d.status;
    a.stats = d.stats;
    a.lkeys = d.lkeys;
    a.lext = d.lext;
    a.lcap = d.lcap;
    a.lcount = d.lcount;
    a.present = d.present;
    a.present_mask = d.present_words ? d.present_words - 1 : 0;
    a.present_hash = d.present_hash;
    return a;
}

// pass-1 item: reads [j*rpt, (j+1)*rpt) of one set, staged in LDS
// The wave's list cursor `cur` persists across the items of one set: entries
// of a chunk it never fills keep the hole mark the launch wrote into the
// whole extension array, so nothing has to be closed at item end.
template <int KW, bool CHECKED>
__device__ void item_pass1(const PassArgs &a, int32_t rpt, int64_t j, uint64_t *s_b2, uint64_t *s_nm,
                           uint64_t *s_hq, ListCursor &cur) {
    const int L = a.read_len, k = a.k, W = L - k + 1;
    const int64_t r0 = j * rpt;
    const int64_t r1 = min(r0 + (int64_t)rpt, a.n_reads);
    // the item's reads are staged in LDS kTileBases bases at a time (read_len <= kTileBases - 64, checked
    // by the host, so a staged run plus its 64-base alignment fits the tile arrays)
    const int64_t sub = kTileBases / L;
    Stats st = {};
    for (int64_t s0 = r0; s0 < r1; s0 += sub) {
        const int64_t s1 = min(s0 + sub, r1);
        if (s0 != r0) __syncthreads();  // the previous run's readers are done
        const int64_t base0 = s0 * L, base1 = s1 * L;
        const int64_t org = base0 & ~(int64_t)63;
        const int64_t mw0 = org >> 6;
        const int nmw = (int)(((base1 + 63) >> 6) - mw0) + 2;
        for (int i = threadIdx.x; i < nmw; i += kBlock) {
            s_nm[i] = a.nm[mw0 + i];
            s_hq[i] = a.hq[mw0 + i];
        }
        for (int i = threadIdx.x; i < 2 * nmw; i += kBlock) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        const Words w{s_b2, s_nm, s_hq};
        const int total = (int)(s1 - s0) * W;
        for (int f0 = 0; f0 < total; f0 += kBlock) {
            if (aborted(a.status)) break;
            const int f = f0 + threadIdx.x;
            Occ o{0, 0, 4, 4};
            bool act = false;
            if (f < total) {
                const int r = f / W;
                const int pos = f - r * W;
                const int64_t rb = (s0 + r) * L - org;
                act = extract(w, rb + pos, rb, rb + L, k, a.forward_only, a.n_owners, a.owner, o);
            }
            pass1_occ<KW, CHECKED>(a, act, o, cur, st);
        }
    }
    (void)st;  // per-item event counters are not collected in the batched form
}

// pass-2 item: first-occurrence entries [j*E, (j+1)*E) of one set
template <int KW, bool CHECKED>
__device__ void item_pass2(const PassArgs &a, int64_t j, int64_t E) {
    if (__hip_atomic_load(a.status, RLX, AGT) & kAbortBits) return;
    const uint64_t n = min((uint64_t)__hip_atomic_load(a.lcount, RLX, AGT), a.lcap);
    const uint64_t b = (uint64_t)j * E, e = min(b + (uint64_t)E, n);
    Stats st = {};
    for (uint64_t i0 = b; i0 < e; i0 += kBlock) {
        const uint64_t i = i0 + threadIdx.x;
        if (i >= e) continue;
        const uint8_t x = a.lext[i];
        if (x == kHole) continue;
        pass2_entry<KW, CHECKED>(a, a.lkeys[2 * i], a.lkeys[2 * i + 1], x, st);
    }
    (void)st;  // per-item event counters are not collected in the batched form
}

// classify + export item: slots [j*SI, (j+1)*SI) of one set, 512-slot chunks
// per wave, classes computed from the counters.
template <int KW>
__device__ void item_export(const BatchHeader *hdr, const BatchDesc &d, int64_t j, int64_t SI, uint16_t *rank_of) {
    hm_export_t out = d.out;
    out.min_depth = hdr->min_depth;
    out.ext_min = hdr->ext_min;
    const uint32_t flags = hdr->export_flags | HM_EXPORT_CLASSIFY;
    const uint64_t b = (uint64_t)j * SI, e = min(b + (uint64_t)SI, d.capacity);
    uint64_t dsum = 0, dxor = 0;
    for (uint64_t first = b + (threadIdx.x >> 6) * (uint64_t)kExportChunk; first < e;
         first += (kBlock / 64) * (uint64_t)kExportChunk)
        export_chunk<KW>(d.slots, first, e, flags, out, d.status, rank_of, dsum, dxor);
    digest_flush(out, dsum, dxor);
}

// Classify + export every set (after the persistent kernel): one block per
// slot range, ranges of all sets concatenated.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_export_batch(const BatchHeader *hdr, const BatchDesc *sets,
                                                         const int64_t *export_start) {
    __shared__ uint16_t s_rank[kBlock / 64][kExportChunk];
    const int S = hdr->n_sets;
    const int64_t total = export_start[S];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int s = __builtin_amdgcn_readfirstlane(find_range(export_start, S, t));
        item_export<KW>(hdr, sets[s], t - export_start[s], hdr->slots_per_item, s_rank[threadIdx.x >> 6]);
    }
}

// Eight waves per SIMD, as the plain pass-1 kernel: both passes' values fit
// the 64-register budget once the set descriptors are constant loads.
template <int KW, bool CHECKED>
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_batch(BatchHeader *hdr, const BatchDesc *sets, const int64_t *item_start,
                                                  const int32_t *group, uint32_t *done) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    __shared__ int64_t s_item;
    __shared__ int s_ok;
    const int S = hdr->n_sets;
    const int64_t n_items = hdr->n_items;
    ListCursor cur{0, kListChunk};
    int cur_set = -1;
    while (true) {
        __syncthreads();  // previous item fully done (LDS, s_item)
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(&hdr->ticket, 1ull);
        __syncthreads();
        // the ticket is block-uniform: keep it (and all per-set descriptor loads) in scalar registers
        const int64_t t = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)s_item >> 32))
                                     << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)s_item));
        if (t >= n_items) break;
        const int g = __builtin_amdgcn_readfirstlane(find_range(item_start, kPhases * S, t));
        const int gs = __builtin_amdgcn_readfirstlane(group[g]);
        const int phase = gs >> 24, s = gs & 0xFFFFFF;
        const int64_t j = t - item_start[g];
        const BatchDesc &d = sets[s];
        if (phase > 0) {
            // acquire: wait until every item of the previous phase of this set is done
            if (threadIdx.x == 0) {
                const uint32_t need = (uint32_t)d.n_items[phase - 1];
                uint32_t *cnt = done + (phase - 1) * S + s;
                const uint64_t t0 = wall_clock64();
                int ok = 1;
                while (__hip_atomic_load(cnt, RLX, AGT) < need) {
                    __builtin_amdgcn_s_sleep(8);
                    if (wall_clock64() - t0 > kWaitTicks) {
                        ok = 0;
                        atomicOr(d.status, HM_ST_TIMEOUT);
                        break;
                    }
                }
                // one agent-scope acquire per block (on this GPU it invalidates the XCD's L2);
                // the barrier below orders the other threads' reads after it
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_ok = ok;
            }
            __syncthreads();
            if (s_ok) item_pass2<KW, CHECKED>(pass_args(hdr, d), j, hdr->list_per_item);
        } else {
            const PassArgs a = pass_args(hdr, d);
            if (s != cur_set) {  // new set: start a fresh chunk (the old one's tail stays marked as holes)
                cur = ListCursor{0, kListChunk};
                cur_set = s;
            }
            item_pass1<KW, CHECKED>(a, d.rpt, j, s_b2, s_nm, s_hq, cur);
        }
        // release: the barrier orders every thread's writes of this item before
        // thread 0's release add, so one agent-scope release (an L2 write-back
        // on this GPU) per item publishes them, not one per wave
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(done + phase * S + s, 1u, __ATOMIC_RELEASE, AGT);
    }
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

size_t hm_batch_work_bytes(int32_t n_sets) { return n_sets > 0 ? layout(n_sets).total : 0; }

int hm_batch_prepare(const hm_batch_set_t *sets, int32_t n_sets, const hm_params_t *p, uint8_t qual_offset,
                     uint8_t qcut, uint32_t export_flags, const hm_batch_tuning_t *tuning, void *work,
                     size_t work_bytes, hm_batch_plan_t *plan, hipStream_t stream) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    if (!sets || n_sets <= 0 || n_sets > (1 << 20)) return fail(HM_EINVAL, "batch: need 1..2^20 sets");
    if (!tuning || !plan || !work) return fail(HM_EINVAL, "batch: tuning, plan and work are required");
    const Layout lay = layout(n_sets);
    if (work_bytes < lay.total) return fail(HM_EINVAL, "batch: work needs %zu bytes", lay.total);
    if ((uintptr_t)work & 255) return fail(HM_EINVAL, "batch: work must be 256-byte aligned");
    const hm_batch_tuning_t tu = *tuning;
    if (tu.blocks_per_cu < 1 || tu.blocks_per_cu > 16) return fail(HM_EINVAL, "batch: blocks_per_cu 1..16");
    if (tu.tile_bases < 1024 || tu.tile_bases > 16 * kTileBases) return fail(HM_EINVAL, "batch: tile_bases 1024..262144");
    if (tu.list_per_item < 256) return fail(HM_EINVAL, "batch: list_per_item >= 256");
    if (tu.slots_per_item < 2048 || tu.slots_per_item % 2048) return fail(HM_EINVAL, "batch: slots_per_item % 2048");
    if (export_flags & ~(HM_EXPORT_UU_ONLY | HM_EXPORT_ALL)) return fail(HM_EINVAL, "batch: unknown export flags");
    if (tu.set_major < 0 || tu.set_major > 64) return fail(HM_EINVAL, "batch: set_major must be 0..64");
    const bool bypass = (p->flags & HM_BLOOM_BYPASS) || p->min_depth == 1;
    const bool in_table = (p->flags & HM_BLOOM_IN_TABLE) != 0;

    std::vector<BatchDesc> descs(n_sets);
    std::vector<int32_t> order(n_sets);
    for (int32_t i = 0; i < n_sets; ++i) {
        const hm_batch_set_t &x = sets[i];
        order[i] = i;
        if (x.n_reads < 0) return fail(HM_EINVAL, "batch set %d: n_reads < 0", i);
        if (x.n_reads > 0 && (x.read_len <= 0 || x.read_len > kTileBases - 64))
            return fail(HM_EINVAL, "batch set %d: read_len must be 1..%d", i, kTileBases - 64);
        if (x.read_len > tu.tile_bases)
            return fail(HM_EINVAL, "batch set %d: read_len exceeds tuning.tile_bases", i);
        if (x.n_reads > 0 && (!x.ascii || !x.qual)) return fail(HM_EINVAL, "batch set %d: reads are NULL", i);
        if (!x.bases2 || !x.nmask || !x.hqmask) return fail(HM_EINVAL, "batch set %d: packed buffers are NULL", i);
        const hm_table_t &t = x.table;
        if (!t.slots || !t.status || !pow2(t.capacity) || ((uintptr_t)t.slots & 63))
            return fail(HM_EINVAL, "batch set %d: bad table", i);
        if (t.k != p->k) return fail(HM_EINVAL, "batch set %d: table k %d != %d", i, t.k, p->k);
        if (!bypass) {
            if (x.bloom.n_hash < 1 || x.bloom.n_hash > 8 ||
                (!in_table && (!x.bloom.words || !pow2(x.bloom.n_words) || x.bloom.n_words > (1ull << 40))))
                return fail(HM_EINVAL, "batch set %d: bad Bloom filter", i);
            if (!x.list.keys || !x.list.ext || !x.list.count) return fail(HM_EINVAL, "batch set %d: bad list", i);
        }
        const hm_export_t &o = x.out;
        if (!o.n_out || (o.capacity > 0 && (!o.key_hi || !o.key_lo || !o.count || !o.tl || !o.tr || !o.cls_l ||
                                            !o.cls_r)))
            return fail(HM_EINVAL, "batch set %d: bad export buffers", i);
        BatchDesc &d = descs[i];
        memset(&d, 0, sizeof d);
        d.ascii = x.ascii;
        d.qual = x.qual;
        d.b2 = x.bases2;
        d.nm = x.nmask;
        d.hq = x.hqmask;
        d.n_reads = x.n_reads;
        d.read_len = x.read_len;
        d.n_bases = x.n_reads * (int64_t)x.read_len;
        d.n_mask_words = hm_mask_words(d.n_bases);
        d.rpt = x.read_len > 0 ? tu.tile_bases / x.read_len : 1;
        if (d.rpt < 1) d.rpt = 1;
        d.slots = reinterpret_cast<Slot *>(t.slots);
        d.capacity = t.capacity;
        const uint64_t mp = t.max_probe ? (uint64_t)t.max_probe : (uint64_t)kDefaultMaxProbe;
        d.max_probe = (uint32_t)(mp < t.capacity ? mp : t.capacity);
        d.status = t.status;
        d.stats = reinterpret_cast<unsigned long long *>(t.stats);
        if (!bypass) {
            d.bloom = in_table ? nullptr : x.bloom.words;  // no pointer: the bits live in the table
            d.bloom_mask = in_table ? 0 : x.bloom.n_words - 1;
            d.n_hash = x.bloom.n_hash;
            d.lkeys = x.list.keys;
            d.lext = x.list.ext;
            d.lcap = x.list.capacity;
            d.lcount = reinterpret_cast<unsigned long long *>(x.list.count);
            if (x.list.present) {
                if (!pow2(x.list.present_words) || x.list.present_hash < 1 || x.list.present_hash > 8)
                    return fail(HM_EINVAL, "batch set %d: bad presence filter", i);
                d.present = x.list.present;
                d.present_words = x.list.present_words;
                d.present_hash = x.list.present_hash;
            }
        }
        d.out = o;
        const bool windows = x.n_reads > 0 && x.read_len >= p->k;
        d.n_items[0] = windows ? (x.n_reads + d.rpt - 1) / d.rpt : 0;
        d.n_items[1] = bypass ? 0 : (int64_t)((d.lcap + tu.list_per_item - 1) / tu.list_per_item);
        d.n_export_items = (int64_t)((t.capacity + tu.slots_per_item - 1) / tu.slots_per_item);
    }
    // larger sets first within every phase
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return descs[a].n_bases > descs[b].n_bases; });
    std::vector<BatchDesc> sorted(n_sets);
    for (int32_t i = 0; i < n_sets; ++i) sorted[i] = descs[order[i]];

    std::vector<uint8_t> blob(lay.total, 0);
    BatchHeader hdr;
    memset(&hdr, 0, sizeof hdr);
    hdr.n_sets = n_sets;
    hdr.k = p->k;
    hdr.forward_only = (p->flags & HM_FORWARD_ONLY) ? 1 : 0;
    hdr.n_owners = p->n_owners;
    hdr.owner = p->owner;
    hdr.bypass = bypass ? 1 : 0;
    hdr.min_depth = p->min_depth;
    hdr.ext_min = p->ext_min;
    hdr.export_flags = export_flags;
    hdr.checked = (p->flags & HM_CHECKED) ? 1 : 0;
    hdr.qual_offset = qual_offset;
    hdr.qcut = qcut;
    hdr.list_per_item = tu.list_per_item;
    hdr.slots_per_item = tu.slots_per_item;
    hdr.seed = p->seed;
    int64_t *item_start = reinterpret_cast<int64_t *>(blob.data() + lay.item_start);
    // ticket order: phase-major (set_major == 0), or set by set with each set's
    // pass 2 placed after the pass 1 of the set_major-th following set, so a
    // pass-2 item rarely has to wait for the tail of its set's pass 1
    int32_t *group = reinterpret_cast<int32_t *>(blob.data() + lay.group);
    std::vector<int32_t> seq;
    if (tu.set_major == 0) {
        for (int ph = 0; ph < kPhases; ++ph)
            for (int32_t i = 0; i < n_sets; ++i) seq.push_back((ph << 24) | i);
    } else {
        const int lag = tu.set_major - 1;
        for (int32_t i = 0; i < n_sets + lag; ++i) {
            if (i < n_sets) seq.push_back(i);                         // pass 1 of set i
            if (i - lag >= 0) seq.push_back((1 << 24) | (i - lag));  // pass 2 of set i - lag
        }
    }
    int64_t acc = 0;
    for (size_t gi = 0; gi < seq.size(); ++gi) {
        item_start[gi] = acc;
        group[gi] = seq[gi];
        acc += sorted[seq[gi] & 0xFFFFFF].n_items[seq[gi] >> 24];
    }
    item_start[kPhases * n_sets] = acc;
    hdr.n_items = acc;
    int64_t *pack_start = reinterpret_cast<int64_t *>(blob.data() + lay.pack_start);
    int64_t pw = 0;
    for (int32_t i = 0; i < n_sets; ++i) {
        pack_start[i] = pw;
        pw += (int64_t)sorted[i].n_mask_words;
    }
    pack_start[n_sets] = pw;
    int64_t *export_start = reinterpret_cast<int64_t *>(blob.data() + lay.export_start);
    int64_t ex = 0;
    for (int32_t i = 0; i < n_sets; ++i) {
        export_start[i] = ex;
        ex += sorted[i].n_export_items;
    }
    export_start[n_sets] = ex;
    Region *reg = reinterpret_cast<Region *>(blob.data() + lay.regions);
    int64_t nr = 0;
    for (int32_t i = 0; i < n_sets; ++i) {
        const BatchDesc &d = sorted[i];
        reg[nr++] = Region{d.slots, d.capacity * HM_SLOT_BYTES, 0u, 0u};
        reg[nr++] = Region{d.bloom, (bypass || !d.bloom) ? 0ull : (d.bloom_mask + 1) * 8, 0u, 0u};
        reg[nr++] = Region{d.lcount, bypass ? 0ull : 8ull, 0u, 0u};
        reg[nr++] = Region{d.lext, bypass ? 0ull : d.lcap, 0xFFFFFFFFu, 0u};  // all holes, exactly lcap bytes
        reg[nr++] = Region{d.present, (bypass || !d.present) ? 0ull : d.present_words * 8, 0u, 0u};
        reg[nr++] = Region{d.out.n_out, 8, 0u, 0u};
        reg[nr++] = Region{d.out.digest, d.out.digest ? 16ull : 0ull, 0u, 0u};
        reg[nr++] = Region{d.status, 4, 0u, 0u};
        reg[nr++] = Region{d.stats, d.stats ? 8ull * HM_N_STATS : 0ull, 0u, 0u};
    }
    // the ticket (inside the header); the per-set phase counters are cleared by hm_batch_launch
    reg[nr++] = Region{reinterpret_cast<uint8_t *>(work) + offsetof(BatchHeader, ticket), 16, 0u, 0u};
    memcpy(blob.data(), &hdr, sizeof hdr);
    memcpy(blob.data() + lay.desc, sorted.data(), sizeof(BatchDesc) * n_sets);
    hipError_t e = hipMemcpyAsync(work, blob.data(), lay.total, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "batch: copy descriptors");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "batch: synchronize");
    plan->work = work;
    plan->n_sets = n_sets;
    plan->grid = device_cus() * tu.blocks_per_cu;
    plan->n_items = acc;
    plan->n_regions = nr;
    plan->pack_words = pw;
    plan->k = p->k;
    plan->reserved = hdr.checked;
    return HM_OK;
}

int hm_batch_launch(const hm_batch_plan_t *plan, hipStream_t s) {
    if (!plan || !plan->work || plan->n_sets <= 0 || plan->grid <= 0) return fail(HM_EINVAL, "batch: bad plan");
    const Layout lay = layout(plan->n_sets);
    uint8_t *w = reinterpret_cast<uint8_t *>(plan->work);
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(w);
    const BatchDesc *descs = reinterpret_cast<const BatchDesc *>(w + lay.desc);
    const int64_t *item_start = reinterpret_cast<const int64_t *>(w + lay.item_start);
    const int32_t *group = reinterpret_cast<const int32_t *>(w + lay.group);
    const int64_t *pack_start = reinterpret_cast<const int64_t *>(w + lay.pack_start);
    const Region *regions = reinterpret_cast<const Region *>(w + lay.regions);
    uint32_t *done = reinterpret_cast<uint32_t *>(w + lay.done);
    // 1. clear (regions, then the phase counters)
    hipLaunchKernelGGL(k_fill_regions, dim3(64, (unsigned)plan->n_regions), dim3(kBlock), 0, s, regions);
    HM_LAUNCH_CHECK("batch: clear");
    int rc = fill<uint32_t>(done, (uint64_t)kPhases * plan->n_sets, 0u, s);
    if (rc) return rc;
    // 2. pack every set
    if (plan->pack_words > 0) {
        hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)grid_for((uint64_t)plan->pack_words, 16)), dim3(kBlock), 0, s,
                           hdr, descs, pack_start);
        HM_LAUNCH_CHECK("batch: pack");
    }
    // 3. the persistent kernel
    if (plan->n_items > 0) {
        const bool checked = plan->reserved != 0;
        const dim3 g((unsigned)plan->grid), b(kBlock);
        if (plan->k >= 32) {
            if (checked) hipLaunchKernelGGL((k_batch<2, true>), g, b, 0, s, hdr, descs, item_start, group, done);
            else hipLaunchKernelGGL((k_batch<2, false>), g, b, 0, s, hdr, descs, item_start, group, done);
        } else {
            if (checked) hipLaunchKernelGGL((k_batch<1, true>), g, b, 0, s, hdr, descs, item_start, group, done);
            else hipLaunchKernelGGL((k_batch<1, false>), g, b, 0, s, hdr, descs, item_start, group, done);
        }
        HM_LAUNCH_CHECK("batch: persistent kernel");
    }
    // 4. classify + export every set
    const int64_t *export_start = reinterpret_cast<const int64_t *>(w + lay.export_start);
    const dim3 ge((unsigned)(device_cus() * 8)), be(kBlock);
    if (plan->k >= 32) hipLaunchKernelGGL(k_export_batch<2>, ge, be, 0, s, hdr, descs, export_start);
    else hipLaunchKernelGGL(k_export_batch<1>, ge, be, 0, s, hdr, descs, export_start);
    HM_LAUNCH_CHECK("batch: export");
    return HM_OK;
}

}  // extern "C"
