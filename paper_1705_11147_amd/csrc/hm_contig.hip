// Contig generation from the UU k-mers (section "Parallel contig
// generation"): the de Bruijn graph of the UU k-mers is a set of simple paths
// and cycles, and every contig is one of them, spelled.
//
// The paper walks the graph from seeds, one walker per seed, and settles two
// walkers that meet with remote atomics.  This is the data-parallel form of
// the same result:
//   1. index: an open-addressing table of 32-byte slots (tag and record
//      number, key, classes) maps a key to its record in one random read;
//   2. link: every UU k-mer looks up its right and left neighbours and keeps
//      a link only where it agrees from both ends and is not a hairpin.  A
//      half-node is a k-mer read in one orientation (2i: key orientation,
//      2i+1: reverse complement); each half-node gets its successor (with the
//      base the step adds) and predecessor, so each path or cycle of k-mers
//      appears twice, once per reading direction (once with HM_FORWARD_ONLY);
//   3. segments (sparse ruling set): chain heads and one k-mer in 32 (picked
//      by a hash of its record number) are rulers; each ruler walks its
//      segment up to the next ruler, once to count it and once to copy its
//      half-nodes and bases into a run of their own; pointer jumping over the
//      rulers alone gives each segment its chain head and rank.  A ruler whose
//      distance passes the number of k-mers sits on a cycle, and so does a
//      half-node that no segment holds;
//   4. cycles (per half-node): pointer jumping gives each cycle half-node the
//      cycle's smallest key; the cycle is cut before it (the reading that
//      holds that k-mer in key orientation becomes a chain, the mirror one a
//      chain that is dropped) and ranked again;
//   5. choose: of the two readings of a path, the one whose first k-mer is
//      smaller is kept: the two spellings are reverse complements of each
//      other and their first k bases already differ, so this is the smaller
//      string;
//   6. spell: each kept chain takes its contig number and base offset from
//      one packed counter (so offsets rise with the contig number); each
//      segment copies its run of bases to its rank, in order.
// Counters shared by the whole grid are updated once per workgroup, not per
// wave, on the paths every k-mer takes.  The round kernels read their work
// counts from device memory, so the whole call is a fixed sequence of
// launches with no host synchronization.
#include "hm_device.h"

namespace hm {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;       // no link / chain end
constexpr uint32_t kInactive = 0xFFFFFFFEu;   // pred of a half-node outside the graph
constexpr uint32_t kCut = 0xFFFFFFFDu;        // pred of a cycle cut's head
constexpr uint32_t kIdMask = 0x3FFFFFFFu;     // successor word: half-node id | added base << 30
constexpr unsigned long long kEmpty = ~0ull;  // empty index slot
constexpr uint64_t kNoOff = ~0ull;            // chain not written
constexpr uint64_t kIndexSeed = 0x13198A2E03707344ull;
constexpr int kRounds = 32;                   // bound on pointer-jumping rounds per phase
constexpr uint32_t kDone = 0x80000000u;       // ruler distance word: rank final
constexpr uint32_t kCycW = 0x7FFFFFFFu;       // ruler distance word: on a cycle
constexpr uint32_t kListDone = 0x80000000u;   // ruler list entry: ranked
constexpr uint32_t kSegEnd = 0x80000000u;     // segment length word: the segment ends its chain
constexpr int kRulerShift = 27;               // 1 ruler in 2^(32 - 27) = 32 k-mers
constexpr int kCntBits = 29;                  // contig counter: number in the high 29 bits,
constexpr int kOffBits = 35;                  // bases in the low 35
constexpr uint64_t kOffMask = (1ull << kOffBits) - 1;
constexpr uint64_t kMaxRecords = 1ull << 29;
// fewer than 2^29 contigs, and at most 2^29 k-mers plus 62 bases per contig
static_assert(kCntBits + kOffBits == 64 && (1ull << kCntBits) >= kMaxRecords, "contig counter fields");
// with fewer than kMaxRecords records a half-node id is at most 2 * kMaxRecords - 3, below kIdMask, so a
// successor word never reads as kNone
static_assert(2 * kMaxRecords - 3 < kIdMask, "half-node ids fit the successor word");
constexpr uint32_t kStop = HM_ST_DUPLICATE | HM_ST_TABLE_FULL;
constexpr int kRulerBuf = 4096;               // workgroup-local ruler buffer (entries)
constexpr int kPer = 16;                      // consecutive entries per thread in the placement passes

struct Ctl {
    unsigned long long alloc;     // (contigs << 35) | bases
    unsigned long long seg_total; // half-nodes placed in segments
    unsigned long long n_cyc;     // half-nodes found on cycles
    unsigned int n_uu;            // UU records
    unsigned int n_rulers;
    unsigned int cnt_re[kRounds + 1];
};
constexpr size_t kCtlBytes = 512;
static_assert(sizeof(Ctl) <= kCtlBytes, "control block");

struct IndexSlot {
    unsigned long long tagj;  // (hash tag << 32) | record, or kEmpty
    uint64_t hi, lo;          // key
    uint64_t cls;             // cls_l | cls_r << 8
};
static_assert(sizeof(IndexSlot) == 32, "index slot");

struct Layout {
    uint64_t slots, half;
    size_t ctl, table, S, RS, hoff, succ, pred, hlen, listA, cyc, rlA, seg, seglen, segoff, visited, total;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Work buffer: control block, index, and arrays of one entry per reading of a
// k-mer (a ruler list entry, a segment position and a cycle list entry also
// number at most that).  The second list of the cycle re-ranking lives in
// hlen until the chains are chosen.
Layout layout(uint64_t cap) {
    Layout L;
    L.slots = ((2 * cap < 64 ? 64 : 2 * cap) + 3) & ~3ull;  // whole 128-byte lines of four slots
    L.half = 2 * cap;
    size_t o = 0;
    L.ctl = o;     o += up256(kCtlBytes);
    L.table = o;   o += up256(L.slots * sizeof(IndexSlot));
    L.S = o;       o += up256(L.half * 8);
    L.RS = o;      o += up256(L.half * 8);
    L.hoff = o;    o += up256(L.half * 8);
    L.succ = o;    o += up256(L.half * 4);
    L.pred = o;    o += up256(L.half * 4);
    L.hlen = o;    o += up256(L.half * 4);
    L.listA = o;   o += up256(L.half * 4);
    L.cyc = o;     o += up256(L.half * 4);
    L.rlA = o;     o += up256(L.half * 4);
    L.seg = o;     o += up256(L.half * 4);
    L.seglen = o;  o += up256(L.half * 4);
    L.segoff = o;  o += up256(L.half * 4);
    L.visited = o; o += up256(L.half);
    L.total = o;
    return L;
}

struct Graph {
    const uint64_t *hi, *lo;
    const uint8_t *cl, *cr;
    const uint64_t *n_out;
    uint64_t cap;
    IndexSlot *table;
    uint64_t slots;
    unsigned long long *S;   // cycle half-nodes: (min node << 32) | ancestor, then (distance << 32) | ancestor
    unsigned long long *RS;  // per ruler: (distance << 32) | ancestor ruler
    uint64_t *hoff;          // per chain head: output offset, or kNoOff
    uint32_t *succ;          // successor id | base it adds << 30, or kNone
    uint32_t *pred, *hlen, *listA, *listB, *cyc, *rlA;
    uint32_t *seg;             // segment runs: half-node id | the base it adds << 30
    uint32_t *seglen, *segoff; // per ruler entry: run length | kSegEnd, run start
    uint8_t *visited;
    Ctl *ctl;
    uint32_t *status;
    int k;
    int fwd;
};

__device__ __forceinline__ uint64_t n_records(const Graph &g) {
    const uint64_t n = *g.n_out;
    return n < g.cap ? n : g.cap;
}

__device__ __forceinline__ bool stopped(const Graph &g) { return (*(volatile uint32_t *)g.status & kStop) != 0; }

__device__ __forceinline__ unsigned long long ld(const unsigned long long *p) {
    return __hip_atomic_load(p, RLX, AGT);
}
__device__ __forceinline__ void st(unsigned long long *p, unsigned long long v) { __hip_atomic_store(p, v, RLX, AGT); }
__device__ __forceinline__ unsigned long long pack(uint32_t hi, uint32_t lo) {
    return ((unsigned long long)hi << 32) | lo;
}

typedef unsigned __int128 u128;

__device__ __forceinline__ u128 key_of(const Graph &g, uint32_t i) { return ((u128)g.hi[i] << 64) | g.lo[i]; }

__device__ __forceinline__ u128 rc128(u128 x, int k) {
    const U128 r = revcomp(U128{(uint64_t)(x >> 64), (uint64_t)x}, k);
    return ((u128)r.hi << 64) | r.lo;
}

// the k-mer of half-node h, as a 2k-bit value read in its orientation
__device__ __forceinline__ u128 seq_of(const Graph &g, uint32_t h) {
    const u128 x = key_of(g, h >> 1);
    return (h & 1) ? rc128(x, g.k) : x;
}

// both readings of a sampled k-mer are rulers
__device__ __forceinline__ bool sampled(uint32_t h) { return ((h >> 1) * 0x9E3779B1u) >> kRulerShift == 0; }

__device__ __forceinline__ uint64_t home_slot(uint64_t h, uint64_t slots) { return __umul64hi(h, slots); }

// Slot of step t of the index's probe sequence from home slot h: the four
// slots of the home slot's 128-byte line (from h on, wrapping within the
// line), then the following lines' slots in order (slots is a multiple of 4).
__device__ __forceinline__ uint64_t index_slot(uint64_t h, uint64_t t, uint64_t slots) {
    if (t < 4) return (h & ~3ull) | ((h + t) & 3);
    const uint64_t w = (h & ~3ull) + t;
    return w >= slots ? w - slots : w;
}

// wave-wide append for rare events: every lane of the wave calls it; lanes
// with `take` get consecutive slots (one atomic per wave that has any)
__device__ __forceinline__ void wave_append(bool take, uint32_t v, uint32_t *list, unsigned int *cnt) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned int base = 0;
    if (lane == leader) base = atomicAdd(cnt, (unsigned int)__popcll(m));
    base = __shfl(base, leader);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1))] = v;
}

// A key lookup in the index: the first slot is loaded by the caller (so two
// lookups can be in flight at once), further slots here.
struct Lookup {
    uint64_t khi, klo, s, home;
    uint32_t tag;
};

__device__ __forceinline__ Lookup lookup_start(const Graph &g, u128 key) {
    Lookup L;
    L.khi = (uint64_t)(key >> 64);
    L.klo = (uint64_t)key;
    const uint64_t h = key_hash(L.khi, L.klo, kIndexSeed);
    L.tag = (uint32_t)(h >> 32);
    L.s = L.home = home_slot(h, g.slots);
    return L;
}

__device__ __forceinline__ void load_slot(const Graph &g, uint64_t s, uint4 &a, uint4 &b) {
    const uint4 *q = reinterpret_cast<const uint4 *>(g.table + s);
    a = q[0];
    b = q[1];
}

// 1: found (record, classes), 0: absent, -1: another key, probe on
__device__ __forceinline__ int slot_match(const Lookup &L, const uint4 &a, const uint4 &b, uint32_t &j, int &cl,
                                          int &cr) {
    const uint64_t tagj = ((uint64_t)a.y << 32) | a.x;
    if (tagj == kEmpty) return 0;
    if ((uint32_t)(tagj >> 32) == L.tag && (((uint64_t)a.w << 32) | a.z) == L.khi &&
        (((uint64_t)b.y << 32) | b.x) == L.klo) {
        j = (uint32_t)tagj;
        cl = (int)(b.z & 0xFF);
        cr = (int)((b.z >> 8) & 0xFF);
        return 1;
    }
    return -1;
}

// record of a key whose first slot (a, b) did not settle it, or kNone
__device__ __forceinline__ uint32_t lookup_rest(const Graph &g, Lookup L, int &cl, int &cr) {
    for (uint64_t p = 1; p < g.slots; ++p) {
        L.s = index_slot(L.home, p, g.slots);
        uint4 a, b;
        load_slot(g, L.s, a, b);
        uint32_t j;
        const int m = slot_match(L, a, b, j, cl, cr);
        if (m >= 0) return m ? j : kNone;
    }
    return kNone;
}

__device__ __forceinline__ bool is_uu(const Graph &g, uint64_t i) { return g.cl[i] < 4 && g.cr[i] < 4; }

// sum of v over the workgroup (every thread calls it; thread 0 gets the sum)
__device__ __forceinline__ unsigned int block_sum(unsigned int v, unsigned int *s_tmp) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
    if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned int t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) t += s_tmp[w];
    return t;
}

// last base of a k-mer read in orientation o (the base a step onto it adds)
__device__ __forceinline__ uint32_t last_base(uint64_t hi, uint64_t lo, int o, int k) {
    if (!o) return (uint32_t)(lo & 3);
    const u128 x = ((u128)hi << 64) | lo;
    return 3u - (uint32_t)((x >> (2 * (k - 1))) & 3);  // the complement of the key's first base
}

// Workgroup placement: each thread brings `mine` (a count, or packed counts),
// the workgroup takes its range of `counter` with one atomic, and each thread
// gets the start of its own part, in thread order.  Every thread of the
// workgroup calls it, the same number of times.
__device__ __forceinline__ unsigned long long block_place(unsigned long long mine, unsigned long long *counter,
                                                          unsigned long long *s_w, unsigned long long *s_base) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    unsigned long long x = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            const unsigned long long v = s_w[w];
            s_w[w] = t;
            t += v;
        }
        *s_base = t ? atomicAdd(counter, t) : 0ull;
    }
    __syncthreads();
    const unsigned long long r = *s_base + s_w[wave] + x - mine;
    __syncthreads();  // s_w and s_base are reused by the next call
    return r;
}

// ------------------------------------------------------------------ 1. index

__global__ __launch_bounds__(kBlock) void k_ctg_index(Graph g) {
    __shared__ unsigned int s_tmp[kBlock / 64];
    const uint64_t n = n_records(g);
    unsigned int n_uu = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
        if (!is_uu(g, i)) continue;
        ++n_uu;
        const uint64_t khi = g.hi[i], klo = g.lo[i];
        const uint64_t h = key_hash(khi, klo, kIndexSeed);
        const uint32_t tag = (uint32_t)(h >> 32);
        const unsigned long long mine = ((unsigned long long)tag << 32) | (uint32_t)i;
        const uint64_t home = home_slot(h, g.slots);
        bool placed = false;
        for (uint64_t p = 0; p < g.slots; ++p) {
            const uint64_t s = index_slot(home, p, g.slots);
            unsigned long long e = g.table[s].tagj;  // a load first: a CAS on a taken slot costs more
            if (e == kEmpty) {
                e = atomicCAS(&g.table[s].tagj, kEmpty, mine);
                if (e == kEmpty) {
                    g.table[s].hi = khi;
                    g.table[s].lo = klo;
                    g.table[s].cls = (uint64_t)g.cl[i] | ((uint64_t)g.cr[i] << 8);
                    placed = true;
                    break;
                }
            }
            if ((uint32_t)(e >> 32) == tag) {
                const uint32_t j = (uint32_t)e;  // compared through the input records (the slot may be half-written)
                if (g.hi[j] == khi && g.lo[j] == klo) {
                    atomicOr(g.status, HM_ST_DUPLICATE);
                    placed = true;
                    break;
                }
            }
        }
        if (!placed) atomicOr(g.status, HM_ST_TABLE_FULL);
    }
    const unsigned int t = block_sum(n_uu, s_tmp);
    if (threadIdx.x == 0 && t) atomicAdd(&g.ctl->n_uu, t);
}

// ------------------------------------------------------------------ 2. link

// The k-mer a step from (i, key orientation) to the right (dir 0) or to the
// left (dir 1) reaches, as the key to look up, its orientation, and the base
// the step drops.
struct Step {
    u128 key;
    int o, drop;
};

__device__ __forceinline__ Step step_target(const Graph &g, u128 s, int cl, int cr, int dir) {
    const int k = g.k;
    const u128 mask = ((u128)1 << (2 * k)) - 1;
    u128 t;
    Step r;
    if (dir == 0) {
        t = ((s << 2) | (u128)cr) & mask;
        r.drop = (int)(s >> (2 * (k - 1))) & 3;
    } else {
        t = (s >> 2) | ((u128)cl << (2 * (k - 1)));
        r.drop = (int)(s & 3);
    }
    r.o = 0;
    r.key = t;
    if (!g.fwd) {
        const u128 rc = rc128(t, k);
        if (rc < t) {
            r.key = rc;
            r.o = 1;
        }
    }
    return r;
}

// The half-node the step reaches, or kNone: the neighbour must be a UU k-mer
// whose extension on the facing side spells the base this k-mer drops, and a
// step back onto the side it left (only possible onto i itself) is no link.
__device__ __forceinline__ uint32_t step_link(uint32_t i, const Step &st_, int dir, uint32_t j, int jl, int jr) {
    if (j == kNone) return kNone;
    // the neighbour's extension facing back, read in its orientation
    const int back = dir == 0 ? (st_.o ? 3 - jr : jl) : (st_.o ? 3 - jl : jr);
    if (back != st_.drop) return kNone;
    if (j == i && st_.o == 1) return kNone;  // hairpin: back onto the side it left
    return 2 * j + (uint32_t)st_.o;
}

// Links of every record; collects the rulers (heads and sampled half-nodes)
// into listA through a wave-local buffer in LDS, flushed with one atomic per
// kRulerBuf / 4 - 128 entries (no workgroup barrier in the loop).
__global__ __launch_bounds__(kBlock) HM_EIGHT_WAVES void k_ctg_link(Graph g) {
    constexpr int kWaveBuf = kRulerBuf / (kBlock / 64);
    __shared__ uint32_t s_buf[kRulerBuf];
    if (stopped(g)) return;
    const uint64_t n = n_records(g);
    const int lane = __lane_id();
    uint32_t *wbuf = s_buf + (threadIdx.x >> 6) * kWaveBuf;
    uint32_t cnt = 0;  // wave-uniform
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t wb = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {  // per wave
        const uint64_t i = wb + lane;
        bool r0 = false, r1 = false;
        uint32_t h0 = 0, h1 = 0;
        if (i < n) {
            h0 = (uint32_t)(2 * i);
            h1 = h0 + 1;
            if (!is_uu(g, i)) {
                g.succ[h0] = g.succ[h1] = kNone;
                g.pred[h0] = g.pred[h1] = kInactive;
            } else {
                const int cl = g.cl[i], cr = g.cr[i];
                const u128 s = key_of(g, (uint32_t)i);
                const Step sr = step_target(g, s, cl, cr, 0), sl = step_target(g, s, cl, cr, 1);
                const Lookup lr = lookup_start(g, sr.key), ll = lookup_start(g, sl.key);
                uint4 ar, br, al, bl;
                load_slot(g, lr.s, ar, br);  // both first probes in flight together
                load_slot(g, ll.s, al, bl);
                // the right and left neighbours: record and classes
                uint32_t jR = kNone, jL = kNone;
                int r_cl = 0, r_cr = 0, l_cl = 0, l_cr = 0;
                int m = slot_match(lr, ar, br, jR, r_cl, r_cr);
                if (m < 0) jR = lookup_rest(g, lr, r_cl, r_cr);
                else if (m == 0) jR = kNone;
                m = slot_match(ll, al, bl, jL, l_cl, l_cr);
                if (m < 0) jL = lookup_rest(g, ll, l_cl, l_cr);
                else if (m == 0) jL = kNone;
                const uint32_t R = step_link((uint32_t)i, sr, 0, jR, r_cl, r_cr);
                const uint32_t Lf = step_link((uint32_t)i, sl, 1, jL, l_cl, l_cr);
                // a successor word carries the base the step adds: the last base of the
                // neighbour read in the walk's direction, which is the right extension
                // (the left step, walked in the reverse-complement reading, adds the
                // complement of the left extension)
                g.succ[h0] = R == kNone ? kNone : (R | (uint32_t)cr << 30);
                g.pred[h0] = Lf;
                const bool samp = sampled(h0);
                r0 = Lf == kNone || samp;
                if (g.fwd) {
                    g.succ[h1] = kNone;
                    g.pred[h1] = kInactive;
                } else {
                    // the reverse-complement reading runs the same links backwards
                    const uint32_t p1 = R == kNone ? kNone : (R ^ 1u);
                    const uint32_t s1 = Lf == kNone ? kNone : (Lf ^ 1u);
                    g.succ[h1] = s1 == kNone ? kNone : (s1 | (3u - (uint32_t)cl) << 30);
                    g.pred[h1] = p1;
                    r1 = p1 == kNone || samp;
                }
            }
        }
        const uint64_t m0 = __ballot(r0), m1 = __ballot(r1);
        const uint64_t below = (1ull << lane) - 1;
        if (r0) wbuf[cnt + __popcll(m0 & below)] = h0;
        cnt += (uint32_t)__popcll(m0);
        if (r1) wbuf[cnt + __popcll(m1 & below)] = h1;
        cnt += (uint32_t)__popcll(m1);
        if (cnt > kWaveBuf - 128 || wb + stride >= n) {  // at most 128 more per pass fit before a flush
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            uint32_t base = 0;
            if (lane == 0 && cnt) base = atomicAdd(&g.ctl->n_rulers, cnt);
            base = __shfl(base, 0);
            for (uint32_t x = lane; x < cnt; x += 64) g.listA[base + x] = wbuf[x];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            cnt = 0;
        }
    }
}

// ------------------------------------------------------------------ 3. segments

// Walk 1: each ruler follows successors up to the next ruler (or its chain's
// end) and records its segment's length (with kSegEnd when the chain ends
// there); the next ruler gets (segment length, this ruler) as its
// ruler-level predecessor, and a head is its own ruler-level head at
// distance 0.  A workgroup owns a contiguous range of the ruler list and a
// lane whose walk ends takes the next one, so no lane idles while the longest
// segment of its wave is walked.
__global__ __launch_bounds__(kBlock) void k_ctg_seglen(Graph g) {
    __shared__ unsigned int s_next;
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_rulers;
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    if (threadIdx.x == 0) s_next = lo + kBlock;
    __syncthreads();
    const uint32_t bound = (uint32_t)(2 * g.cap);
    uint32_t x = lo + threadIdx.x, R = 0, cur = 0, t = 0;
    bool live = x < hi;
    if (live) {
        R = cur = g.listA[x];
        if (g.pred[R] == kNone) st(g.RS + R, pack(0, R));
    }
    while (live) {
        const uint32_t w = g.succ[cur];
        const uint32_t nx = w & kIdMask;
        bool end = w == kNone || sampled(nx);
        if (!end && ++t >= bound) {  // longer than the graph: cannot happen
            atomicOr(g.status, HM_ST_TIMEOUT);
            end = true;
            t = 0;
        } else if (!end) {
            cur = nx;
        }
        if (end) {
            if (w != kNone) st(g.RS + nx, pack(t + 1, R));
            g.seglen[x] = (t + 1) | (w == kNone ? kSegEnd : 0u);
            x = atomicAdd(&s_next, 1u);
            live = x < hi;
            if (live) {
                R = cur = g.listA[x];
                t = 0;
                if (g.pred[R] == kNone) st(g.RS + R, pack(0, R));
            }
        }
    }
}

// Each ruler entry's run in the segment arrays, kPer consecutive entries per
// thread, one atomic per workgroup.
__global__ __launch_bounds__(kBlock) void k_ctg_segplace(Graph g) {
    __shared__ unsigned long long s_w[kBlock / 64], s_base;
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_rulers;
    const uint32_t chunk = kBlock * kPer;
    for (uint32_t c0 = blockIdx.x * chunk; c0 < n; c0 += gridDim.x * chunk) {  // uniform per workgroup
        const uint32_t x0 = c0 + threadIdx.x * kPer;
        unsigned long long mine = 0;
        for (int j = 0; j < kPer && x0 + j < n; ++j) mine += g.seglen[x0 + j] & ~kSegEnd;
        unsigned long long at = block_place(mine, &g.ctl->seg_total, s_w, &s_base);
        for (int j = 0; j < kPer && x0 + j < n; ++j) {
            g.segoff[x0 + j] = (uint32_t)at;
            at += g.seglen[x0 + j] & ~kSegEnd;
        }
    }
}

// Walk 2: each ruler copies its segment into its run: each half-node's id with
// the base it adds, which is the successor word that reached it (the ruler's
// own base: the last base of its k-mer).  A lane stages its entries in LDS and
// writes each 64-byte block of its run at once (one entry per step of the walk
// would leave each line half written between the walk's random reads).
constexpr uint32_t kStage = 16;  // entries of a 64-byte block of a run

// Stage entry w at run position p; the staged entries are positions
// p + 1 - nb .. p of one run, written out at the end of a block or of the run.
__device__ __forceinline__ void stage_put(uint32_t *seg, uint32_t *stage, uint32_t &nb, uint32_t p, uint32_t w,
                                          bool last) {
    stage[nb++] = w;
    if (((p + 1) & (kStage - 1)) == 0 || last) {
        const uint32_t first = p + 1 - nb;
        if (nb == kStage) {  // a whole aligned block
            uint4 *d = reinterpret_cast<uint4 *>(seg + first);
            for (uint32_t q = 0; q < kStage / 4; ++q)
                d[q] = make_uint4(stage[4 * q], stage[4 * q + 1], stage[4 * q + 2], stage[4 * q + 3]);
        } else {
            for (uint32_t q = 0; q < nb; ++q) seg[first + q] = stage[q];
        }
        nb = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_ctg_segfill(Graph g) {
    __shared__ unsigned int s_next;
    __shared__ uint32_t s_stage[kBlock * (kStage + 1)];
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_rulers;
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    if (threadIdx.x == 0) s_next = lo + kBlock;
    __syncthreads();
    uint32_t *stage = s_stage + threadIdx.x * (kStage + 1);
    const uint64_t room = 2 * g.cap;
    uint32_t x = lo + threadIdx.x, cur = 0, t = 0, len = 0, o = 0, nb = 0;
    bool live = x < hi;
    bool fresh = live;  // x is a new ruler entry: place its ruler first
    while (live) {
        if (fresh) {
            fresh = false;
            const uint32_t R = g.listA[x] & ~kListDone;
            len = g.seglen[x] & ~kSegEnd;
            o = g.segoff[x];
            t = 0;
            nb = 0;
            cur = R;
            if ((uint64_t)o + len > room || len == 0) {  // more than the graph holds, or empty: cannot happen
                atomicOr(g.status, HM_ST_TIMEOUT);
                len = 0;
            } else {
                const uint32_t b = last_base(g.hi[R >> 1], g.lo[R >> 1], (int)(R & 1), g.k);
                stage_put(g.seg, stage, nb, o, R | b << 30, len == 1);
            }
        } else if (t + 1 < len) {
            const uint32_t w = g.succ[cur];
            if (w == kNone) {  // shorter than walk 1 found it: cannot happen
                atomicOr(g.status, HM_ST_TIMEOUT);
                len = 0;
                nb = 0;
                continue;
            }
            cur = w & kIdMask;
            ++t;
            stage_put(g.seg, stage, nb, o + t, w, t + 1 == len);
        } else {
            x = atomicAdd(&s_next, 1u);
            live = x < hi;
            fresh = live;
        }
    }
}

// One round of pointer jumping over the rulers: a ruler whose ancestor is a
// head (or already ranked) is ranked; the others take their ancestor's
// ancestor; a distance past the number of UU k-mers marks a cycle.  Enough
// rounds for both run: ceil(log2(UU k-mers + 1)) + 2.
__global__ __launch_bounds__(kBlock) void k_ctg_rjump(Graph g, int r) {
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_rulers;
    const uint32_t limit = g.ctl->n_uu + 1u;
    const int rounds = (32 - __clz(limit - 1u)) + 2;
    if (n == 0 || r >= rounds) return;
    const uint32_t half = (uint32_t)(2 * g.cap);
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const uint32_t e = g.listA[x];
        if (e & kListDone) continue;
        const unsigned long long v = ld(g.RS + e);
        const uint32_t J = (uint32_t)v, W = (uint32_t)(v >> 32);
        if (J >= half) {  // a ruler no walker reached: cannot happen
            atomicOr(g.status, HM_ST_TIMEOUT);
            g.listA[x] = e | kListDone;
            continue;
        }
        const unsigned long long v2 = ld(g.RS + J);
        const uint32_t J2 = (uint32_t)v2, W2r = (uint32_t)(v2 >> 32), W2 = W2r & ~kDone;
        bool settled = true;
        if (W2r == kCycW) {
            st(g.RS + e, pack(kCycW, J2));
        } else if (J2 == J && W2 == 0) {
            st(g.RS + e, pack(W | kDone, J));  // J is the head
        } else {
            const uint32_t w = W + W2;
            if (W2r & kDone) {
                st(g.RS + e, pack(w | kDone, J2));  // J2 is the head
            } else if (w >= limit) {
                st(g.RS + e, pack(kCycW, J2));
            } else {
                st(g.RS + e, pack(w, J2));
                settled = false;
            }
        }
        if (settled) g.listA[x] = e | kListDone;
    }
}

// The half-nodes of cycle rulers' segments go to the cycle list (kPer ruler
// entries per thread, one atomic per workgroup).
__global__ __launch_bounds__(kBlock) void k_ctg_cycseg(Graph g) {
    __shared__ unsigned long long s_w[kBlock / 64], s_base;
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_rulers;
    const uint32_t chunk = kBlock * kPer;
    for (uint32_t c0 = blockIdx.x * chunk; c0 < n; c0 += gridDim.x * chunk) {  // uniform per workgroup
        const uint32_t x0 = c0 + threadIdx.x * kPer;
        unsigned long long mine = 0;
        for (int j = 0; j < kPer && x0 + j < n; ++j) {
            const uint32_t R = g.listA[x0 + j] & ~kListDone;
            if ((uint32_t)(ld(g.RS + R) >> 32) == kCycW) mine += g.seglen[x0 + j] & ~kSegEnd;
        }
        unsigned long long at = block_place(mine, &g.ctl->n_cyc, s_w, &s_base);
        if (!mine) continue;
        for (int j = 0; j < kPer && x0 + j < n; ++j) {
            const uint32_t R = g.listA[x0 + j] & ~kListDone;
            if ((uint32_t)(ld(g.RS + R) >> 32) != kCycW) continue;
            const uint32_t len = g.seglen[x0 + j] & ~kSegEnd, o = g.segoff[x0 + j];
            for (uint32_t t = 0; t < len; ++t) g.cyc[at + t] = g.seg[o + t] & kIdMask;
            at += len;
        }
    }
}

// Half-nodes that no segment holds sit on cycles without a ruler.  These
// three kernels find them, and return at once when the segments hold every
// half-node of the graph (the usual case).
__device__ __forceinline__ bool all_placed(const Graph &g) {
    const unsigned long long active = (unsigned long long)g.ctl->n_uu * (g.fwd ? 1u : 2u);
    return g.ctl->seg_total >= active;
}

__global__ __launch_bounds__(kBlock) void k_ctg_visit_clear(Graph g) {
    if (stopped(g) || all_placed(g)) return;
    const uint64_t nh = 2 * n_records(g);
    for (uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x; h < nh; h += (uint64_t)gridDim.x * kBlock)
        g.visited[h] = 0;
}

__global__ __launch_bounds__(kBlock) void k_ctg_visit_mark(Graph g) {
    if (stopped(g) || all_placed(g)) return;
    const uint64_t np = g.ctl->seg_total;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < np; p += (uint64_t)gridDim.x * kBlock)
        g.visited[g.seg[p] & kIdMask] = 1;
}

__global__ __launch_bounds__(kBlock) void k_ctg_visit_scan(Graph g) {
    __shared__ unsigned long long s_w[kBlock / 64], s_base;
    if (stopped(g) || all_placed(g)) return;
    const uint64_t nh = 2 * n_records(g);
    const uint64_t chunk = (uint64_t)kBlock * kPer;
    for (uint64_t c0 = (uint64_t)blockIdx.x * chunk; c0 < nh; c0 += (uint64_t)gridDim.x * chunk) {  // uniform
        const uint64_t h0 = c0 + (uint64_t)threadIdx.x * kPer;
        uint32_t bits = 0;
        for (int j = 0; j < kPer && h0 + j < nh; ++j)
            if (g.pred[h0 + j] != kInactive && !g.visited[h0 + j]) bits |= 1u << j;
        unsigned long long at = block_place((unsigned long long)__popc(bits), &g.ctl->n_cyc, s_w, &s_base);
        for (int j = 0; j < kPer; ++j)
            if ((bits >> j) & 1) g.cyc[at++] = (uint32_t)(h0 + j);
    }
}

// One round of pointer jumping over the half-nodes of the cut cycles (rlA and
// listB alternate): a half-node whose ancestor is a head is done, the others
// take their ancestor's ancestor.  Rounds past the last non-empty one find a
// zero count and return.
__global__ __launch_bounds__(kBlock) void k_ctg_jump(Graph g, int r) {
    if (stopped(g)) return;
    unsigned int *cnt = g.ctl->cnt_re;
    const uint32_t n = __hip_atomic_load(cnt + r, RLX, AGT);
    if (n == 0) return;
    const uint32_t *in = (r & 1) ? g.listB : g.rlA;
    uint32_t *out = (r & 1) ? g.rlA : g.listB;
    const uint32_t limit = g.ctl->n_uu + 1u;
    const int lane = __lane_id();
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t wb = blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {
        const uint32_t idx = wb + lane;
        bool more = false;
        uint32_t h = 0;
        if (idx < n) {
            h = in[idx];
            const unsigned long long v = ld(g.S + h);
            const uint32_t J = (uint32_t)v, W = (uint32_t)(v >> 32);
            const unsigned long long v2 = ld(g.S + J);
            const uint32_t J2 = (uint32_t)v2, W2 = (uint32_t)(v2 >> 32);
            if (!(J2 == J && W2 == 0)) {
                const uint32_t w = W + W2;
                st(g.S + h, pack(w, J2));
                more = w < limit;
                if (!more) atomicOr(g.status, HM_ST_TIMEOUT);  // no cycle is left after the cuts: cannot happen
            }
        }
        wave_append(more, h, out, cnt + r + 1);
    }
}

// ------------------------------------------------------------------ 4. cycles

__global__ __launch_bounds__(kBlock) void k_ctg_cyc_init(Graph g) {
    if (stopped(g)) return;
    const uint32_t n = (uint32_t)g.ctl->n_cyc;
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const uint32_t h = g.cyc[x];
        uint32_t p = g.pred[h];
        if (p >= 2 * g.cap) {  // a cycle half-node has a predecessor: cannot happen
            atomicOr(g.status, HM_ST_TIMEOUT);
            p = h;
        }
        st(g.S + h, pack(h >> 1, p));  // window (pred, h]: its smallest node is h's
    }
}

// One round of min-jumping on the cycle half-nodes: the window behind each
// one doubles (at least), so after ceil(log2(cycle half-nodes)) rounds it
// spans its whole cycle and holds the node of the cycle's smallest key.
__global__ __launch_bounds__(kBlock) void k_ctg_cyc_jump(Graph g, int r) {
    if (stopped(g)) return;
    const uint32_t n = (uint32_t)g.ctl->n_cyc;
    if (n <= 1) return;
    const int rounds = 32 - __clz(n - 1);
    if (r >= rounds) return;
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const uint32_t h = g.cyc[x];
        const unsigned long long v = ld(g.S + h);
        const uint32_t J = (uint32_t)v, M = (uint32_t)(v >> 32);
        const unsigned long long v2 = ld(g.S + J);
        const uint32_t J2 = (uint32_t)v2, M2 = (uint32_t)(v2 >> 32);
        const uint32_t m = (M2 != M && key_of(g, M2) < key_of(g, M)) ? M2 : M;
        st(g.S + h, pack(m, J2));
    }
}

// Cut each directed cycle before its smallest node: that half-node becomes a
// head (marked kCut) and its predecessor a tail; the others start ranking
// again from their predecessor.
__global__ __launch_bounds__(kBlock) void k_ctg_cut(Graph g) {
    if (stopped(g)) return;
    const uint32_t n = (uint32_t)g.ctl->n_cyc;
    const int lane = __lane_id();
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t wb = blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {
        const uint32_t x = wb + lane;
        bool more = false;
        uint32_t h = 0;
        if (x < n) {
            h = g.cyc[x];
            const uint32_t M = (uint32_t)(ld(g.S + h) >> 32);
            const uint32_t p = g.pred[h];
            if (p >= 2 * g.cap) {
                atomicOr(g.status, HM_ST_TIMEOUT);  // not on a cycle after all: cannot happen
            } else if ((h >> 1) == M) {
                st(g.S + h, pack(0, h));
                g.pred[h] = kCut;
                g.succ[p] = kNone;
            } else {
                st(g.S + h, pack(1, p));
                more = true;
            }
        }
        wave_append(more, h, g.rlA, &g.ctl->cnt_re[0]);
    }
}

// ------------------------------------------------------------------ 5. choose

// At every chain end: keep the chain or not, and give its head the chain's
// length.  Entries x < n_rulers are ruler entries (a path segment that ends
// its chain); the rest are cycle half-nodes (the tail left by a cut).
__global__ __launch_bounds__(kBlock) void k_ctg_choose(Graph g) {
    if (stopped(g)) return;
    const uint32_t nr = g.ctl->n_rulers, n = nr + (uint32_t)g.ctl->n_cyc;
    const uint32_t half = (uint32_t)(2 * g.cap);
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        if (x < nr) {
            const uint32_t sl = g.seglen[x];
            if (!(sl & kSegEnd)) continue;
            const uint32_t R = g.listA[x] & ~kListDone;
            const unsigned long long v = ld(g.RS + R);
            const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
            if (W == kCycW || !(W & kDone) || H >= half) continue;  // a cycle's, or not ranked (reported)
            const uint32_t len = sl & ~kSegEnd;
            const uint32_t tail = g.seg[g.segoff[x] + len - 1] & kIdMask;
            const uint32_t last = (W & ~kDone) + len - 1;  // the tail's rank
            const bool keep = g.fwd || seq_of(g, H) < seq_of(g, tail ^ 1u);
            g.hlen[H] = keep ? last + 1 : 0;
        } else {
            const uint32_t t = g.cyc[x - nr];
            if (g.succ[t] != kNone) continue;
            const unsigned long long v = ld(g.S + t);
            const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
            if (H >= half || g.pred[H] != kCut) continue;  // not ranked (reported): cannot happen
            g.hlen[H] = (H & 1) == 0 ? W + 1 : 0;  // the cycle read from its smallest key, key orientation
        }
    }
}

// ------------------------------------------------------------------ 6. spell

// The chain head of entry x (a path head among the rulers, a cut head among
// the cycle half-nodes), or kNone.
__device__ __forceinline__ uint32_t head_of_entry(const Graph &g, uint32_t x, uint32_t nr) {
    if (x < nr) {
        const uint32_t R = g.listA[x] & ~kListDone;
        return g.pred[R] == kNone ? R : kNone;
    }
    const uint32_t h = g.cyc[x - nr];
    return g.pred[h] == kCut ? h : kNone;
}

// Contig numbers and offsets: kPer entries per thread; a workgroup sums its
// chains' (1, bases) pairs (packed in one word), takes its range with one
// atomic, and hands the range out in order.
__global__ __launch_bounds__(kBlock) void k_ctg_alloc(Graph g, uint64_t *off, uint64_t off_cap, uint64_t seq_cap) {
    __shared__ unsigned long long s_w[kBlock / 64], s_base;
    if (stopped(g)) return;
    const uint32_t nr = g.ctl->n_rulers, n = nr + (uint32_t)g.ctl->n_cyc;
    const uint32_t chunk = kBlock * kPer;
    for (uint32_t c0 = blockIdx.x * chunk; c0 < n; c0 += gridDim.x * chunk) {  // uniform per workgroup
        const uint32_t x0 = c0 + threadIdx.x * kPer;
        unsigned long long mine = 0;
        for (int j = 0; j < kPer && x0 + j < n; ++j) {
            const uint32_t H = head_of_entry(g, x0 + j, nr);
            if (H == kNone) continue;
            const uint32_t len = g.hlen[H];
            if (len) mine += (1ull << kOffBits) | ((uint64_t)g.k + len - 1);
        }
        unsigned long long at = block_place(mine, &g.ctl->alloc, s_w, &s_base);
        for (int j = 0; j < kPer && x0 + j < n; ++j) {
            const uint32_t H = head_of_entry(g, x0 + j, nr);
            if (H == kNone) continue;
            const uint32_t len = g.hlen[H];
            uint64_t o = kNoOff;
            if (len) {
                const uint64_t bases = (uint64_t)g.k + len - 1;
                const uint64_t c = at >> kOffBits, b = at & kOffMask;
                if (c < off_cap) off[c] = b;
                if (c < off_cap && b + bases <= seq_cap) o = b;
                else atomicOr(g.status, HM_ST_OUTPUT_FULL);
                at += (1ull << kOffBits) | bases;
            }
            g.hoff[H] = o;
        }
    }
}

__device__ __forceinline__ void write_kmer(uint8_t *seq, uint64_t o, u128 s, int k) {
    for (int b = k - 1; b >= 0; --b) {
        seq[o + b] = (uint8_t)"ACGT"[(int)(s & 3)];
        s >>= 2;
    }
}

// Spell the kept chains: a path segment copies its run of bases to its rank
// (the head writes its whole k-mer), in order; a cycle half-node writes its
// base at its rank.  Path segments go 64 to a wave: each lane finds one
// segment's place, then the whole wave copies the 64 runs one after the
// other, its lanes on consecutive bases, so the loads and stores coalesce.
__global__ __launch_bounds__(kBlock) void k_ctg_write(Graph g, uint8_t *seq, uint64_t seq_cap) {
    if (stopped(g)) return;
    const uint32_t nr = g.ctl->n_rulers, n = nr + (uint32_t)g.ctl->n_cyc;
    const uint32_t half = (uint32_t)(2 * g.cap);
    const int k = g.k;
    const int lane = __lane_id();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t x0 = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * 64u; x0 < nr; x0 += waves * 64u) {
        const uint32_t x = x0 + lane;
        unsigned long long dst = kNoOff;  // where the run's first base goes, or kNoOff: nothing to write
        uint32_t len = 0, s0 = 0, t0 = 0;
        if (x < nr) {
            const uint32_t R = g.listA[x] & ~kListDone;
            const unsigned long long v = ld(g.RS + R);
            const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
            if (W != kCycW && (W & kDone) && H < half) {
                const uint64_t o = g.hoff[H];  // kNoOff for a dropped chain
                const uint32_t rank = W & ~kDone;
                len = g.seglen[x] & ~kSegEnd;
                s0 = g.segoff[x];
                if (o < seq_cap && (uint64_t)k + rank + len - 1 <= seq_cap - o) {  // else past the room: cannot happen
                    if (rank == 0) {  // the head's segment starts with the head's k-mer
                        write_kmer(seq, o, seq_of(g, H), k);
                        t0 = 1;
                    }
                    dst = o + k - 1 + rank;
                }
            }
        }
        for (int j = 0; j < 64; ++j) {  // wave-uniform
            const unsigned long long d = __shfl(dst, j);
            if (d == kNoOff) continue;
            const uint32_t lj = __shfl(len, j), sj = __shfl(s0, j);
            for (uint32_t t = __shfl(t0, j) + lane; t < lj; t += 64) seq[d + t] = (uint8_t)"ACGT"[g.seg[sj + t] >> 30];
        }
    }
    for (uint32_t x = nr + blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const uint32_t h = g.cyc[x - nr];
        const unsigned long long v = ld(g.S + h);
        const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
        if (H >= half) continue;
        const uint64_t o = g.hoff[H];
        if (o >= seq_cap || (uint64_t)k + W > seq_cap - o) continue;  // kNoOff, or past the room
        const u128 s = seq_of(g, h);
        if (W == 0) write_kmer(seq, o, s, k);
        else seq[o + k - 1 + W] = (uint8_t)"ACGT"[(int)(s & 3)];
    }
}

__global__ void k_ctg_final(Graph g, uint64_t *counts, uint64_t *off, uint64_t off_cap, uint64_t seq_cap) {
    if (threadIdx.x != 0) return;
    const unsigned long long a = g.ctl->alloc;
    const uint64_t nc = a >> kOffBits, nb = a & kOffMask;
    counts[0] = nc;
    counts[1] = nb;
    if (g.ctl->cnt_re[kRounds]) atomicOr(g.status, HM_ST_TIMEOUT);
    if (nc <= off_cap) off[nc] = nb;
    if (nc > off_cap || nb > seq_cap) atomicOr(g.status, HM_ST_OUTPUT_FULL);
}

int check_contigs(const hm_export_t *uu, int32_t k, uint32_t flags, const hm_contigs_t *out) {
    if (!uu || !out) return fail(HM_EINVAL, "contigs: NULL argument");
    if (k < 1 || k > 63) return fail(HM_EINVAL, "contigs: k must be in 1..63 (got %d)", k);
    if (flags & ~HM_FORWARD_ONLY) return fail(HM_EINVAL, "contigs: unknown flags 0x%x", flags);
    if (!(flags & HM_FORWARD_ONLY) && !(k & 1))
        return fail(HM_EINVAL, "contigs: k must be odd for canonical k-mers (got %d)", k);
    if (uu->capacity >= kMaxRecords) return fail(HM_EINVAL, "contigs: capacity must be below 2^29");
    if (!uu->n_out) return fail(HM_EINVAL, "contigs: n_out is NULL");
    if (uu->capacity && (!uu->key_hi || !uu->key_lo || !uu->cls_l || !uu->cls_r))
        return fail(HM_EINVAL, "contigs: record arrays are NULL");
    if (!out->counts || !out->status || !out->off) return fail(HM_EINVAL, "contigs: counts, status or off is NULL");
    if (out->seq_capacity && !out->seq) return fail(HM_EINVAL, "contigs: seq is NULL");
    if (!out->work || (reinterpret_cast<uintptr_t>(out->work) & 255))
        return fail(HM_EINVAL, "contigs: work must be a 256-byte aligned device buffer");
    if (out->work_bytes < layout(uu->capacity).total)
        return fail(HM_EINVAL, "contigs: work holds %llu bytes, %llu needed", (unsigned long long)out->work_bytes,
                    (unsigned long long)layout(uu->capacity).total);
    return HM_OK;
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

size_t hm_contigs_work_bytes(uint64_t capacity) {
    if (capacity >= kMaxRecords) return 0;
    return layout(capacity).total;
}

int hm_contigs(const hm_export_t *uu, int32_t k, uint32_t flags, hm_contigs_t *out, hipStream_t s) {
    int rc = check_contigs(uu, k, flags, out);
    if (rc) return rc;
    const Layout L = layout(uu->capacity);
    char *w = static_cast<char *>(out->work);
    Graph g;
    g.hi = uu->key_hi;
    g.lo = uu->key_lo;
    g.cl = uu->cls_l;
    g.cr = uu->cls_r;
    g.n_out = uu->n_out;
    g.cap = uu->capacity;
    g.table = reinterpret_cast<IndexSlot *>(w + L.table);
    g.slots = L.slots;
    g.S = reinterpret_cast<unsigned long long *>(w + L.S);
    g.RS = reinterpret_cast<unsigned long long *>(w + L.RS);
    g.hoff = reinterpret_cast<uint64_t *>(w + L.hoff);
    g.succ = reinterpret_cast<uint32_t *>(w + L.succ);
    g.pred = reinterpret_cast<uint32_t *>(w + L.pred);
    g.hlen = reinterpret_cast<uint32_t *>(w + L.hlen);
    g.listA = reinterpret_cast<uint32_t *>(w + L.listA);
    g.listB = g.hlen;  // second re-ranking list, free until the chains are chosen
    g.cyc = reinterpret_cast<uint32_t *>(w + L.cyc);
    g.rlA = reinterpret_cast<uint32_t *>(w + L.rlA);
    g.seg = reinterpret_cast<uint32_t *>(w + L.seg);
    g.seglen = reinterpret_cast<uint32_t *>(w + L.seglen);
    g.segoff = reinterpret_cast<uint32_t *>(w + L.segoff);
    g.visited = reinterpret_cast<uint8_t *>(w + L.visited);
    g.ctl = reinterpret_cast<Ctl *>(w + L.ctl);
    g.status = out->status;
    g.k = k;
    g.fwd = (flags & HM_FORWARD_ONLY) ? 1 : 0;
    // clears are fill kernels, so the call can be captured in a graph
    if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(w + L.ctl), kCtlBytes / 4, 0u, s))) return rc;
    if ((rc = fill<uint32_t>(out->status, 1, 0u, s))) return rc;
    if ((rc = fill<uint64_t>(out->counts, 2, 0ull, s))) return rc;
    // empty index: all ones (the tag word marks a slot empty)
    if ((rc = fill<uint4>(reinterpret_cast<uint4 *>(g.table), 2 * L.slots, make_uint4(~0u, ~0u, ~0u, ~0u), s)))
        return rc;
    const uint64_t cap = uu->capacity ? uu->capacity : 1;
    const dim3 blk(kBlock);
    const dim3 g_rec((unsigned)grid_for(cap, 16));
    const dim3 g_half((unsigned)grid_for(2 * cap, 16));
    const dim3 g_rul((unsigned)grid_for(2 * cap / 16 + 1, 16));
    hipLaunchKernelGGL(k_ctg_index, g_rec, blk, 0, s, g);
    HM_LAUNCH_CHECK("hm_contigs (index)");
    hipLaunchKernelGGL(k_ctg_link, g_rec, blk, 0, s, g);
    HM_LAUNCH_CHECK("hm_contigs (link)");
    hipLaunchKernelGGL(k_ctg_seglen, g_rul, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_segplace, g_rul, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_segfill, g_rul, blk, 0, s, g);
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_rjump, g_rul, blk, 0, s, g, r);
    HM_LAUNCH_CHECK("hm_contigs (segments)");
    hipLaunchKernelGGL(k_ctg_cycseg, g_rul, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_visit_clear, g_half, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_visit_mark, g_half, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_visit_scan, g_half, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_cyc_init, g_half, blk, 0, s, g);
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_cyc_jump, g_half, blk, 0, s, g, r);
    hipLaunchKernelGGL(k_ctg_cut, g_half, blk, 0, s, g);
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_jump, g_half, blk, 0, s, g, r);
    HM_LAUNCH_CHECK("hm_contigs (cycles)");
    hipLaunchKernelGGL(k_ctg_choose, g_rul, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_alloc, g_rul, blk, 0, s, g, out->off, out->off_capacity, out->seq_capacity);
    hipLaunchKernelGGL(k_ctg_write, g_rul, blk, 0, s, g, out->seq, out->seq_capacity);
    hipLaunchKernelGGL(k_ctg_final, dim3(1), dim3(64), 0, s, g, out->counts, out->off, out->off_capacity,
                       out->seq_capacity);
    HM_LAUNCH_CHECK("hm_contigs (spell)");
    return HM_OK;
}

}  // extern "C"
