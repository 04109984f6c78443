// Contig generation from the UU k-mers (section "Parallel contig
// generation"): the de Bruijn graph of the UU k-mers is a set of simple paths
// and cycles, and every contig is one of them, spelled.
//
// The paper walks the graph from seeds, one walker per seed, and settles two
// walkers that meet with remote atomics.  This is the data-parallel form of
// the same result:
//   1. index: an open-addressing table maps a key to its record;
//   2. link: every UU k-mer looks up its right and left neighbours (two
//      lookups) and keeps a link only where it agrees from both ends and is
//      not a hairpin.  A half-node is a k-mer read in one orientation
//      (2i: key orientation, 2i+1: reverse complement); each half-node gets
//      its successor and predecessor, so each path or cycle of k-mers appears
//      twice, once per reading direction (once with HM_FORWARD_ONLY);
//   3. rank: pointer jumping over predecessors (in place, a packed (ancestor,
//      distance) word per half-node) gives every half-node its chain head and
//      its rank; a half-node whose distance passes the number of k-mers sits
//      on a cycle;
//   4. cycles: a second pointer jumping gives every cycle half-node the
//      cycle's smallest key; the cycle is cut before it (the reading that
//      holds that k-mer in key orientation becomes a chain, the mirror one a
//      chain that is dropped) and ranked again;
//   5. choose: of the two readings of a path, the one whose first k-mer is
//      smaller is kept: the two spellings are reverse complements of each
//      other and their first k bases already differ, so this is the smaller
//      string;
//   6. spell: each kept chain takes its contig number and base offset from
//      one packed counter (so offsets rise with the contig number), and every
//      half-node writes its base at its rank.
// The round kernels read their work counts from device memory, so the whole
// call is a fixed sequence of launches with no host synchronization.
#include "hm_device.h"

namespace hm {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;      // no link / chain end
constexpr uint32_t kInactive = 0xFFFFFFFEu;  // pred of a half-node outside the graph
constexpr uint32_t kCut = 0xFFFFFFFDu;       // pred of a cycle cut's head
constexpr uint64_t kEmpty = ~0ull;           // empty index slot
constexpr uint64_t kNoOff = ~0ull;           // chain not written
constexpr uint64_t kIndexSeed = 0x13198A2E03707344ull;
constexpr int kRounds = 32;                   // bound on pointer-jumping rounds per phase
constexpr int kCntBits = 29;                  // contig counter: number in the high 29 bits,
constexpr int kOffBits = 35;                  // bases in the low 35
constexpr uint64_t kOffMask = (1ull << kOffBits) - 1;
constexpr uint64_t kMaxRecords = 1ull << 29;
// fewer than 2^29 contigs, and at most 2^29 k-mers plus 62 bases per contig
static_assert(kCntBits + kOffBits == 64 && (1ull << kCntBits) >= kMaxRecords, "contig counter fields");
constexpr uint32_t kStop = HM_ST_DUPLICATE | HM_ST_TABLE_FULL;

struct Ctl {
    unsigned long long alloc;      // (contigs << 35) | bases
    unsigned int n_uu;             // UU records
    unsigned int n_cyc;            // half-nodes found on cycles
    unsigned int cnt_main[kRounds + 1];
    unsigned int cnt_re[kRounds + 1];
};
constexpr size_t kCtlBytes = 512;
static_assert(sizeof(Ctl) <= kCtlBytes, "control block");

struct Layout {
    uint64_t slots, half;
    size_t ctl, table, S, succ, pred, hlen, hoff, listA, listB, cyc, total;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(uint64_t cap) {
    Layout L;
    uint64_t t = 64;
    while (t < 2 * cap) t <<= 1;
    L.slots = t;
    L.half = 2 * cap;
    size_t o = 0;
    L.ctl = o;   o += up256(kCtlBytes);
    L.table = o; o += up256(t * 8);
    L.S = o;     o += up256(L.half * 8);
    L.hoff = o;  o += up256(L.half * 8);
    L.succ = o;  o += up256(L.half * 4);
    L.pred = o;  o += up256(L.half * 4);
    L.hlen = o;  o += up256(L.half * 4);
    L.listA = o; o += up256(L.half * 4);
    L.listB = o; o += up256(L.half * 4);
    L.cyc = o;   o += up256(L.half * 4);
    L.total = o;
    return L;
}

struct Graph {
    const uint64_t *hi, *lo;
    const uint8_t *cl, *cr;
    const uint64_t *n_out;
    uint64_t cap;
    uint64_t *table;
    uint64_t tmask;
    unsigned long long *S;  // (distance << 32) | ancestor; in the cycle phase (min node << 32) | ancestor
    uint64_t *hoff;
    uint32_t *succ, *pred, *hlen, *listA, *listB, *cyc;
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

// wave-wide append: every lane of the wave calls it; lanes with `take` get consecutive slots
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

// slot of a key in the index, or kNone
__device__ __forceinline__ uint32_t find(const Graph &g, u128 key) {
    const uint64_t khi = (uint64_t)(key >> 64), klo = (uint64_t)key;
    const uint64_t h = key_hash(khi, klo, kIndexSeed);
    const uint32_t tag = (uint32_t)(h >> 32);
    uint64_t s = h & g.tmask;
    for (uint64_t p = 0; p <= g.tmask; ++p) {
        const uint64_t e = g.table[s];
        if (e == kEmpty) return kNone;
        if ((uint32_t)(e >> 32) == tag) {
            const uint32_t j = (uint32_t)e;
            if (g.hi[j] == khi && g.lo[j] == klo) return j;
        }
        s = (s + 1) & g.tmask;
    }
    return kNone;
}

__device__ __forceinline__ bool is_uu(const Graph &g, uint64_t i) { return g.cl[i] < 4 && g.cr[i] < 4; }

// ------------------------------------------------------------------ 1. index

__global__ __launch_bounds__(kBlock) void k_ctg_index(Graph g) {
    const uint64_t n = n_records(g);
    const int lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t wb = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {
        const uint64_t i = wb + lane;
        const bool uu = i < n && is_uu(g, i);
        if (uu) {
            const uint64_t khi = g.hi[i], klo = g.lo[i];
            const uint64_t h = key_hash(khi, klo, kIndexSeed);
            const uint32_t tag = (uint32_t)(h >> 32);
            const uint64_t mine = ((uint64_t)tag << 32) | (uint32_t)i;
            uint64_t s = h & g.tmask;
            bool placed = false;
            for (uint64_t p = 0; p <= g.tmask && !placed; ++p) {
                uint64_t e = g.table[s];
                if (e == kEmpty) {
                    e = atomicCAS(reinterpret_cast<unsigned long long *>(g.table + s), (unsigned long long)kEmpty,
                                  (unsigned long long)mine);
                    if (e == kEmpty) {
                        placed = true;
                        break;
                    }
                }
                if ((uint32_t)(e >> 32) == tag) {
                    const uint32_t j = (uint32_t)e;
                    if (g.hi[j] == khi && g.lo[j] == klo) {
                        atomicOr(g.status, HM_ST_DUPLICATE);
                        placed = true;
                        break;
                    }
                }
                s = (s + 1) & g.tmask;
            }
            if (!placed) atomicOr(g.status, HM_ST_TABLE_FULL);
        }
        const uint64_t m = __ballot(uu);
        if (lane == 0 && m) atomicAdd(&g.ctl->n_uu, (unsigned int)__popcll(m));
    }
}

// ------------------------------------------------------------------ 2. link

// Half-node reached by a step from (i, key orientation) to the right (dir 0)
// or to the left (dir 1), or kNone: the neighbour must be a UU k-mer whose
// extension on the facing side spells the base this k-mer drops, and a step
// back onto the side it left (only possible onto i itself) is no link.
__device__ __forceinline__ uint32_t step(const Graph &g, uint32_t i, u128 s, int cl, int cr, int dir) {
    const int k = g.k;
    const u128 mask = ((u128)1 << (2 * k)) - 1;
    u128 t;
    int drop;
    if (dir == 0) {
        t = ((s << 2) | (u128)cr) & mask;
        drop = (int)(s >> (2 * (k - 1))) & 3;
    } else {
        t = (s >> 2) | ((u128)cl << (2 * (k - 1)));
        drop = (int)(s & 3);
    }
    int o = 0;
    u128 key = t;
    if (!g.fwd) {
        const u128 r = rc128(t, k);
        if (r < t) {
            key = r;
            o = 1;
        }
    }
    const uint32_t j = find(g, key);
    if (j == kNone) return kNone;
    // the neighbour's extension facing back, read in its orientation
    int back;
    if (dir == 0) back = o ? 3 - (int)g.cr[j] : (int)g.cl[j];
    else back = o ? 3 - (int)g.cl[j] : (int)g.cr[j];
    if (back != drop) return kNone;
    if (j == i && o == 1) return kNone;  // hairpin: back onto the side it left
    return 2 * j + (uint32_t)o;
}

__global__ __launch_bounds__(kBlock) void k_ctg_link(Graph g) {
    if (stopped(g)) return;
    const uint64_t n = n_records(g);
    const int lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t wb = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {
        const uint64_t i = wb + lane;
        bool in0 = false, in1 = false;
        uint32_t h0 = 0, h1 = 0;
        if (i < n) {
            h0 = (uint32_t)(2 * i);
            h1 = h0 + 1;
            if (!is_uu(g, i)) {
                g.succ[h0] = g.succ[h1] = kNone;
                g.pred[h0] = g.pred[h1] = kInactive;
                st(g.S + h0, pack(0, h0));
                st(g.S + h1, pack(0, h1));
            } else {
                const int cl = g.cl[i], cr = g.cr[i];
                const u128 s = key_of(g, (uint32_t)i);
                const uint32_t R = step(g, (uint32_t)i, s, cl, cr, 0);
                const uint32_t Lf = step(g, (uint32_t)i, s, cl, cr, 1);
                g.succ[h0] = R;
                g.pred[h0] = Lf;
                st(g.S + h0, Lf == kNone ? pack(0, h0) : pack(1, Lf));
                in0 = Lf != kNone;
                if (g.fwd) {
                    g.succ[h1] = kNone;
                    g.pred[h1] = kInactive;
                    st(g.S + h1, pack(0, h1));
                } else {
                    // the reverse-complement reading runs the same links backwards
                    const uint32_t s1 = Lf == kNone ? kNone : (Lf ^ 1u);
                    const uint32_t p1 = R == kNone ? kNone : (R ^ 1u);
                    g.succ[h1] = s1;
                    g.pred[h1] = p1;
                    st(g.S + h1, p1 == kNone ? pack(0, h1) : pack(1, p1));
                    in1 = p1 != kNone;
                }
            }
        }
        wave_append(in0, h0, g.listA, &g.ctl->cnt_main[0]);
        wave_append(in1, h1, g.listA, &g.ctl->cnt_main[0]);
    }
}

// ------------------------------------------------------------------ 3. rank

// One round of pointer jumping over the half-nodes in `in`: a half-node whose
// ancestor is a chain head is done; the others take their ancestor's ancestor
// and move to `out`, or to the cycle list once the distance passes the number
// of UU k-mers (no path is that long).  Rounds past the last non-empty one
// find a zero count and return.
__global__ __launch_bounds__(kBlock) void k_ctg_jump(Graph g, int phase, int r) {
    if (stopped(g)) return;
    unsigned int *cnt = phase == 0 ? g.ctl->cnt_main : g.ctl->cnt_re;
    const uint32_t n = __hip_atomic_load(cnt + r, RLX, AGT);
    if (n == 0) return;
    const uint32_t *in = (r & 1) ? g.listB : g.listA;
    uint32_t *out = (r & 1) ? g.listA : g.listB;
    const uint32_t limit = g.ctl->n_uu + 1u;
    const int lane = __lane_id();
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t wb = blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < n; wb += stride) {
        const uint32_t idx = wb + lane;
        bool more = false, cyc = false;
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
                cyc = w >= limit;
                more = !cyc;
                if (cyc && phase != 0) {  // no cycle is left after the cuts: cannot happen
                    atomicOr(g.status, HM_ST_TIMEOUT);
                    cyc = false;
                }
            }
        }
        wave_append(more, h, out, cnt + r + 1);
        wave_append(cyc, h, g.cyc, &g.ctl->n_cyc);
    }
}

// ------------------------------------------------------------------ 4. cycles

__global__ __launch_bounds__(kBlock) void k_ctg_cyc_init(Graph g) {
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_cyc;
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const uint32_t h = g.cyc[x];
        st(g.S + h, pack(h >> 1, g.pred[h]));  // window (pred, h]: its smallest node is h's
    }
}

// One round of min-jumping on the cycle half-nodes: the window behind each
// one doubles (at least), so after ceil(log2(cycle half-nodes)) rounds it
// spans its whole cycle and holds the node of the cycle's smallest key.
__global__ __launch_bounds__(kBlock) void k_ctg_cyc_jump(Graph g, int r) {
    if (stopped(g)) return;
    const uint32_t n = g.ctl->n_cyc;
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
    const uint32_t n = g.ctl->n_cyc;
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
        wave_append(more, h, g.listA, &g.ctl->cnt_re[0]);
    }
}

// ------------------------------------------------------------------ 5. choose

// At every chain's tail: keep the chain or not, and give its head the length.
__global__ __launch_bounds__(kBlock) void k_ctg_choose(Graph g) {
    if (stopped(g)) return;
    const uint64_t nh = 2 * n_records(g);
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < nh; t += (uint64_t)gridDim.x * kBlock) {
        if (g.pred[t] == kInactive || g.succ[t] != kNone) continue;
        const unsigned long long v = ld(g.S + t);
        const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
        bool keep;
        if (g.pred[H] == kCut) keep = (H & 1) == 0;  // the cycle read from its smallest key, key orientation
        else keep = g.fwd || seq_of(g, H) < seq_of(g, (uint32_t)t ^ 1u);
        g.hlen[H] = keep ? W + 1 : 0;
    }
}

// ------------------------------------------------------------------ 6. spell

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__global__ __launch_bounds__(kBlock) void k_ctg_alloc(Graph g, uint64_t *off, uint64_t off_cap, uint64_t seq_cap) {
    if (stopped(g)) return;
    const uint64_t nh = 2 * n_records(g);
    const int lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t wb = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); wb < nh; wb += stride) {
        const uint64_t h = wb + lane;
        uint64_t bases = 0;
        bool head = false;
        if (h < nh) {
            const uint32_t p = g.pred[h];
            head = p == kNone || p == kCut;
            if (head) {
                const uint32_t len = g.hlen[h];
                if (len) bases = (uint64_t)g.k + len - 1;
            }
        }
        const unsigned long long mine = bases ? ((1ull << kOffBits) | bases) : 0ull;
        const unsigned long long incl = wave_incl_scan(mine);
        const unsigned long long tot = __shfl(incl, 63, 64);
        unsigned long long base = 0;
        if (tot) {
            if (lane == 0) base = atomicAdd(&g.ctl->alloc, tot);
            base = __shfl(base, 0, 64);
        }
        if (head) {
            uint64_t o = kNoOff;
            if (bases) {
                const unsigned long long at = base + incl - mine;
                const uint64_t c = at >> kOffBits, b = at & kOffMask;
                if (c < off_cap) off[c] = b;
                if (c < off_cap && b + bases <= seq_cap) o = b;
                else atomicOr(g.status, HM_ST_OUTPUT_FULL);
            }
            g.hoff[h] = o;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_ctg_write(Graph g, uint8_t *seq, uint64_t seq_cap) {
    if (stopped(g)) return;
    const uint64_t nh = 2 * n_records(g);
    const int k = g.k;
    for (uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x; h < nh; h += (uint64_t)gridDim.x * kBlock) {
        if (g.pred[h] == kInactive) continue;
        const unsigned long long v = ld(g.S + h);
        const uint32_t H = (uint32_t)v, W = (uint32_t)(v >> 32);
        // only a head has an offset (a half-node that did not reach one is
        // reported by k_ctg_final and writes nothing)
        const uint32_t hp = g.pred[H];
        if ((hp != kNone && hp != kCut) || ld(g.S + H) != pack(0, H)) continue;
        const uint64_t o = g.hoff[H];
        if (o == kNoOff || o + k + W > seq_cap) continue;
        u128 s = seq_of(g, (uint32_t)h);
        if (W == 0) {
            for (int b = k - 1; b >= 0; --b) {
                seq[o + b] = (uint8_t)"ACGT"[(int)(s & 3)];
                s >>= 2;
            }
        } else {
            seq[o + k - 1 + W] = (uint8_t)"ACGT"[(int)(s & 3)];
        }
    }
}

__global__ void k_ctg_final(Graph g, uint64_t *counts, uint64_t *off, uint64_t off_cap, uint64_t seq_cap) {
    if (threadIdx.x != 0) return;
    const unsigned long long a = g.ctl->alloc;
    const uint64_t nc = a >> kOffBits, nb = a & kOffMask;
    counts[0] = nc;
    counts[1] = nb;
    if (g.ctl->cnt_main[kRounds] || g.ctl->cnt_re[kRounds]) atomicOr(g.status, HM_ST_TIMEOUT);
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
    g.table = reinterpret_cast<uint64_t *>(w + L.table);
    g.tmask = L.slots - 1;
    g.S = reinterpret_cast<unsigned long long *>(w + L.S);
    g.hoff = reinterpret_cast<uint64_t *>(w + L.hoff);
    g.succ = reinterpret_cast<uint32_t *>(w + L.succ);
    g.pred = reinterpret_cast<uint32_t *>(w + L.pred);
    g.hlen = reinterpret_cast<uint32_t *>(w + L.hlen);
    g.listA = reinterpret_cast<uint32_t *>(w + L.listA);
    g.listB = reinterpret_cast<uint32_t *>(w + L.listB);
    g.cyc = reinterpret_cast<uint32_t *>(w + L.cyc);
    g.ctl = reinterpret_cast<Ctl *>(w + L.ctl);
    g.status = out->status;
    g.k = k;
    g.fwd = (flags & HM_FORWARD_ONLY) ? 1 : 0;
    // clears are fill kernels, so the call can be captured in a graph
    if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(w + L.ctl), kCtlBytes / 4, 0u, s))) return rc;
    if ((rc = fill<uint32_t>(out->status, 1, 0u, s))) return rc;
    if ((rc = fill<uint64_t>(out->counts, 2, 0ull, s))) return rc;
    if ((rc = fill<uint64_t>(g.table, L.slots, kEmpty, s))) return rc;
    const uint64_t cap = uu->capacity ? uu->capacity : 1;
    const dim3 blk(kBlock);
    const dim3 g_rec((unsigned)grid_for(cap, 16));
    const dim3 g_half((unsigned)grid_for(2 * cap, 16));
    hipLaunchKernelGGL(k_ctg_index, g_rec, blk, 0, s, g);
    HM_LAUNCH_CHECK("hm_contigs (index)");
    hipLaunchKernelGGL(k_ctg_link, g_rec, blk, 0, s, g);
    HM_LAUNCH_CHECK("hm_contigs (link)");
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_jump, g_half, blk, 0, s, g, 0, r);
    HM_LAUNCH_CHECK("hm_contigs (rank)");
    hipLaunchKernelGGL(k_ctg_cyc_init, g_half, blk, 0, s, g);
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_cyc_jump, g_half, blk, 0, s, g, r);
    hipLaunchKernelGGL(k_ctg_cut, g_half, blk, 0, s, g);
    for (int r = 0; r < kRounds; ++r) hipLaunchKernelGGL(k_ctg_jump, g_half, blk, 0, s, g, 1, r);
    HM_LAUNCH_CHECK("hm_contigs (cycles)");
    hipLaunchKernelGGL(k_ctg_choose, g_half, blk, 0, s, g);
    hipLaunchKernelGGL(k_ctg_alloc, g_half, blk, 0, s, g, out->off, out->off_capacity, out->seq_capacity);
    hipLaunchKernelGGL(k_ctg_write, g_half, blk, 0, s, g, out->seq, out->seq_capacity);
    hipLaunchKernelGGL(k_ctg_final, dim3(1), dim3(64), 0, s, g, out->counts, out->off, out->off_capacity,
                       out->seq_capacity);
    HM_LAUNCH_CHECK("hm_contigs (spell)");
    return HM_OK;
}

}  // extern "C"
