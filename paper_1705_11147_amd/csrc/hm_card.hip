// hm_card.hip -- the cardinality pass that precedes counting (section
// "Parallel k-mer analysis"): a HyperLogLog estimate of the distinct k-mers,
// which sizes the Bloom filter; an exact count of a hash-sampled subset of
// the keys, which estimates how many k-mers survive the depth filter and so
// sizes the count table; and a sample of windows, whose most frequent keys
// are the heavy hitters.
//
// One kernel visits every window with the same tiling as pass 1.  Each
// workgroup keeps its own copy of the registers in LDS, one byte each.  A
// window raises its register only when its rank is larger than the byte: a
// plain LDS read first, and since registers only grow, almost every window
// stops there once the sketch has warmed up; the rare raise is a
// compare-and-swap on the enclosing 32-bit LDS word.  When the workgroup is
// done it raises the device registers with atomicMax wherever its bytes are
// larger: the register-wise maximum is the merge of two sketches.  The two
// samples are rare events (1 in 2^sample_log2 keys, 1 in 2^heavy_log2
// windows) counted in small open-addressing tables with the pass-1 probe and
// counter code.
#include "hm_bins.h"
#include "hm_roll.h"

namespace hm {
namespace {

constexpr uint64_t kCardSeed = 0xB7E151628AED2A6Aull;  // cardinality hash (definition constant)
constexpr uint64_t kPosSeed = 0x452821E638D01377ull;   // window sampling hash (definition constant)
constexpr int kCardBlocksPerCu = 4;
constexpr int kCardMaxP = 16;
constexpr int kCardHistBlock = 512;  // threads of the pass that also counts the partition's histogram

struct CardArgs {
    uint32_t *regs;
    int p;
    uint64_t smask, hmask;
    Slot *s_slots;
    uint64_t s_cmask;
    uint32_t s_probe;
    uint32_t *s_status;
    Slot *h_slots;
    uint64_t h_cmask;
    uint32_t h_probe;
    uint32_t *h_status;
    unsigned long long *positions;
    uint64_t seed;
};

// Raise byte i of the LDS registers to v (no-op when it is already >= v).
__device__ __forceinline__ void lds_raise(uint8_t *regs, uint32_t i, uint32_t v) {
    if (regs[i] >= v) return;
    uint32_t *w = reinterpret_cast<uint32_t *>(regs + (i & ~3u));
    const uint32_t sh = (i & 3u) * 8;
    uint32_t old = *w;
    while (((old >> sh) & 255u) < v) {
        const uint32_t prev = atomicCAS(w, old, (old & ~(255u << sh)) | (v << sh));
        if (prev == old) break;
        old = prev;
    }
}

// Count one occurrence (no extensions) of a key in a sample table.  Once the
// table is reported full its counts are void, so later samples skip the probe.
template <int KW>
__device__ __forceinline__ void sample_count(Slot *slots, uint64_t cmask, uint32_t max_probe, uint32_t *status,
                                             uint64_t seed, const Occ &o) {
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & HM_ST_TABLE_FULL) return;
    uint64_t A, B;
    slot_words<KW>(o.hi, o.lo, A, B);
    const Probe pr = table_find<KW>(slots, cmask, key_hash(o.hi, o.lo, seed), A, B, max_probe, true);
    if (pr.slot >= 0) count_occurrence<false>(slots + pr.slot, 4, 4, status, pr.narrow);
    else atomicOr(status, HM_ST_TABLE_FULL);
}

template <int KW>
__device__ __forceinline__ void card_window(const CardArgs &c, uint8_t *s_reg, bool act, const Occ &o, int64_t j,
                                            uint32_t &npos) {
    if (!act) return;
    ++npos;
    const uint64_t h = fmix64(fmix64(o.hi ^ kCardSeed) ^ o.lo);
    const uint32_t reg = (uint32_t)(h >> (64 - c.p));
    const uint64_t rest = h << c.p;
    const uint32_t rho = rest ? (uint32_t)__clzll((long long)rest) + 1u : (uint32_t)(65 - c.p);
    lds_raise(s_reg, reg, rho);
    if ((h & c.smask) == 0) sample_count<KW>(c.s_slots, c.s_cmask, c.s_probe, c.s_status, c.seed, o);
    if ((fmix64((uint64_t)j ^ kPosSeed) & c.hmask) == 0)
        sample_count<KW>(c.h_slots, c.h_cmask, c.h_probe, c.h_status, c.seed, o);
}

__device__ __forceinline__ void card_begin(const CardArgs &c, uint32_t *s_reg32) {
    for (int i = threadIdx.x; i < (1 << c.p) / 4; i += blockDim.x) s_reg32[i] = 0;
    __syncthreads();
}

__device__ __forceinline__ void card_end(const CardArgs &c, const uint8_t *s_reg, uint32_t npos) {
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << c.p); i += blockDim.x) {
        const uint32_t v = s_reg[i];
        if (v > c.regs[i]) atomicMax(c.regs + i, v);  // the plain read only skips needless atomics
    }
    uint64_t x = npos;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (lane_id() == 0 && x) atomicAdd(c.positions, (unsigned long long)x);
}

// Fixed-length reads, tiles staged in LDS as in pass 1, but each lane takes a run of kCardRun
// consecutive windows of one read, rolled from one window to the next (Roll, RunBits); the
// extensions are not needed here.

// The first partition level's histogram of the binned path, counted on the way (HIST): the
// number of owned windows of each group in this workgroup's tiles, into
// hist1[blockIdx.x * groups + group] (the layout hm_bin_kmers reads).
struct BinHist {
    uint32_t *hist1;
    int total_bits, bin_bits;
};

template <int KW, bool HIST = false, int NT = kBlock>
__global__ __launch_bounds__(NT) void k_card_fixed(PassArgs a, CardArgs c, int32_t reads_per_tile, int64_t n_tiles,
                                                   BinHist bh) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    extern __shared__ uint32_t s_reg32[];  // 2^p bytes of registers (then, with HIST, the group counters)
    uint8_t *s_reg = reinterpret_cast<uint8_t *>(s_reg32);
    uint32_t *s_g = s_reg32 + ((1 << c.p) >> 2);
    const int ng = HIST ? 1 << (bh.total_bits - bh.bin_bits) : 0;
    for (int i = threadIdx.x; i < ng; i += NT) s_g[i] = 0;
    card_begin(c, s_reg32);
    uint32_t npos = 0;
    const int L = a.read_len, k = a.k;
    const int W = L - k + 1;  // > 0, checked by the host
    const int runs = (W + kCardRun - 1) / kCardRun;
    const typename Roll<KW>::Shape sh = Roll<KW>::shape(k);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t org = (r0 * L) & ~(int64_t)63;
        const int64_t mw0 = org >> 6;
        const int nmw = (int)((((r1 * L) + 63) >> 6) - mw0) + 2;
        __syncthreads();
        for (int i = threadIdx.x; i < nmw; i += NT) s_nm[i] = a.nm[mw0 + i];
        for (int i = threadIdx.x; i < 2 * nmw; i += NT) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        const Words w{s_b2, s_nm, nullptr};
        const int total = (int)(r1 - r0) * runs;
        for (int g = threadIdx.x; g < total; g += NT) {
            const int r = g / runs;
            const int p0 = (g - r * runs) * kCardRun;
            const int cnt = min(kCardRun, W - p0);
            const int64_t j0 = (r0 + r) * L - org + p0;  // first window, relative to the tile origin
            const int64_t jg = (r0 + r) * L + p0;        // and in the read set
            RunBits rb;
            rb.load(w, j0, k);
            const uint32_t vm = rb.valid_mask(k, cnt);
            Roll<KW> x;
            {
                const U128 f = w.window(j0, k);
                x.set(f, revcomp(f, k));
            }
            for (int i = 0; i < cnt; ++i) {
                if (i > 0) x.step((uint32_t)rb.base(i), sh);
                if (!((vm >> i) & 1u)) continue;
                const bool fwd = a.forward_only || x.forward();
                Occ o{fwd ? x.fhi() : x.rhi(), fwd ? x.flo() : x.rlo(), 4, 4};
                if (a.n_owners > 1 && owner_of(o.hi, o.lo, a.n_owners) != a.owner) continue;
                card_window<KW>(c, s_reg, true, o, jg + i, npos);
                if (HIST) atomicAdd(&s_g[bin_of(o.hi, o.lo, bh.total_bits) >> bh.bin_bits], 1u);
            }
        }
    }
    card_end(c, s_reg, npos);  // starts with a barrier: the group counters are complete
    if (HIST)
        for (int i = threadIdx.x; i < ng; i += NT) bh.hist1[(size_t)blockIdx.x * ng + i] = s_g[i];
}

// The same pass over fixed-length reads, also writing every owned occurrence
// to a stream (hm_cardinality_occ) with its extensions, for a pass 1 that
// then reads the stream instead of rescanning every window.  With an owner
// filter a wave holds an owned window in only a few lanes at a time, so the
// owned-window work (HyperLogLog hash and register, samples, extensions,
// stream store) is not done where the window is found: each lane only rolls
// its windows, takes the canonical key and tests the owner, and the owned
// ones are staged in the wave's ring in LDS with their position.  Every 64
// staged windows, and at the end of each tile, the wave finishes them with
// every lane busy.  The loops have wave-uniform trip counts for that (a lane
// past the tile's runs, or past its read's last window, idles).
template <int KW>
__global__ __launch_bounds__(kBlock) void k_card_fixed_occ(PassArgs a, CardArgs c, OccOut out, int32_t reads_per_tile,
                                                           int64_t n_tiles) {
    __shared__ uint64_t s_b2[kTileB2Words];
    __shared__ uint64_t s_nm[kTileMaskWords];
    __shared__ uint64_t s_hq[kTileMaskWords];
    __shared__ uint4 s_rkey[kBlock / 64][kRing];
    __shared__ uint32_t s_raux[kBlock / 64][kRing];
    extern __shared__ uint32_t s_reg32[];  // 2^p bytes of registers
    uint8_t *s_reg = reinterpret_cast<uint8_t *>(s_reg32);
    card_begin(c, s_reg32);
    const int wv = threadIdx.x >> 6;
    OccRing ring{s_rkey[wv], s_raux[wv], 0u, 0u};
    OccCursor cur{0ull, kOccChunk};
    uint32_t npos = 0;
    const int L = a.read_len, k = a.k;
    const int W = L - k + 1;  // > 0, checked by the host
    const int runs = (W + kCardRun - 1) / kCardRun;
    const typename Roll<KW>::Shape sh = Roll<KW>::shape(k);
    // the owner filter's operands, held in a vector register: read from the kernel arguments in
    // the per-window loop they cost a scalar load and a wait on every outstanding LDS store
    uint32_t n_own = a.n_owners, me = a.owner;
    asm volatile("" : "+v"(n_own), "+v"(me));
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile * reads_per_tile;
        const int64_t r1 = min(r0 + (int64_t)reads_per_tile, a.n_reads);
        const int64_t org = (r0 * L) & ~(int64_t)63;
        const int64_t mw0 = org >> 6;
        const int nmw = (int)((((r1 * L) + 63) >> 6) - mw0) + 2;
        __syncthreads();
        for (int i = threadIdx.x; i < nmw; i += kBlock) {
            s_nm[i] = a.nm[mw0 + i];
            s_hq[i] = a.hq[mw0 + i];
        }
        for (int i = threadIdx.x; i < 2 * nmw; i += kBlock) s_b2[i] = a.b2[2 * mw0 + i];
        __syncthreads();
        const Words w{s_b2, s_nm, s_hq};
        // finish the n oldest staged windows (wave-uniform n <= 64), one per lane; aux packs the
        // window's start (tile-relative, 15 bits), its offset in its read (15 bits) and orientation
        auto finish = [&](uint32_t n) {
            uint4 kk = make_uint4(0, 0, 0, 0);
            uint32_t m = 0;
            uint8_t e = 0;
            if (ring_take(ring, n, kk, m)) {
                const int64_t j = m & 0x7FFF;
                const int pos = (int)((m >> 15) & 0x7FFF);
                const bool fwd = (m >> 31) != 0;
                Occ o{((uint64_t)kk.y << 32) | kk.x, ((uint64_t)kk.w << 32) | kk.z, 4, 4};
                card_window<KW>(c, s_reg, true, o, org + j, npos);
                // HQ neighbours inside the read, as pass 1 takes them
                const int lb = (pos > 0 && w.hqbit(j - 1)) ? (int)w.code(j - 1) : 4;
                const int rr = (pos + k < L && w.hqbit(j + k)) ? (int)w.code(j + k) : 4;
                const int left = fwd ? lb : (rr < 4 ? 3 - rr : 4);
                const int right = fwd ? rr : (lb < 4 ? 3 - lb : 4);
                e = (uint8_t)(left | (right << 4));
            }
            occ_emit(out, cur, n, kk, e);
        };
        const int total = (int)(r1 - r0) * runs;
        for (int g0 = 0; g0 < total; g0 += kBlock) {  // workgroup-uniform trip count
            const int gi = g0 + threadIdx.x;
            int p0 = 0;
            int64_t j0 = 0;
            uint32_t vm = 0;  // windows of the lane's run that hold no invalid base (none past its read)
            Roll<KW> x;
            x.set(U128{0, 0}, U128{0, 0});
            RunBits rb{0, 0, 0};
            if (gi < total) {
                const int r = gi / runs;
                p0 = (gi - r * runs) * kCardRun;
                j0 = (r0 + r) * L - org + p0;  // first window of the run, relative to the tile origin
                rb.load(w, j0, k);
                vm = rb.valid_mask(k, min(kCardRun, W - p0));
                const U128 f = w.window(j0, k);
                x.set(f, revcomp(f, k));
            }
#pragma unroll
            for (int i = 0; i < kCardRun; ++i) {
                // every lane rolls (an idle lane's code is never used): no divergent branch
                if (i > 0) x.step((uint32_t)rb.base(i), sh);
                const bool fwd = a.forward_only || x.forward();
                const uint64_t khi = fwd ? x.fhi() : x.rhi(), klo = fwd ? x.flo() : x.rlo();
                const bool act = ((vm >> i) & 1u) && (n_own <= 1 || owner_of(khi, klo, n_own) == me);
                const uint32_t aux = (uint32_t)(j0 + i) | ((uint32_t)(p0 + i) << 15) | (fwd ? 1u << 31 : 0u);
                ring_push(ring, act, khi, klo, aux);
                if (ring.tail - ring.head >= 64) finish(64);
            }
        }
        if (ring.tail != ring.head) finish(ring.tail - ring.head);  // before the next tile replaces the LDS words
    }
    card_end(c, s_reg, npos);
    occ_close(out, cur);
}

template <int KW>
__global__ __launch_bounds__(kBlock) void k_card_var(PassArgs a, CardArgs c, int64_t n_tiles) {
    __shared__ int64_t s_off[kVarReads + 1];
    __shared__ int64_t s_pre[kVarReads + 1];
    extern __shared__ uint32_t s_reg32[];
    uint8_t *s_reg = reinterpret_cast<uint8_t *>(s_reg32);
    card_begin(c, s_reg32);
    uint32_t npos = 0;
    var_windows<false>(a, n_tiles, s_off, s_pre,
                       [&](bool act, const Occ &o, int64_t j) { card_window<KW>(c, s_reg, act, o, j, npos); });
    card_end(c, s_reg, npos);
}

// Variable-length reads, writing the owned occurrences too (extract() gives
// them with their extensions; var_windows' trip counts are workgroup-uniform).
// The sketch is updated where a window is found; the stream entries are
// staged in the wave's ring and written 64 at a time.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_card_var_occ(PassArgs a, CardArgs c, OccOut out, int64_t n_tiles) {
    __shared__ int64_t s_off[kVarReads + 1];
    __shared__ int64_t s_pre[kVarReads + 1];
    __shared__ uint4 s_rkey[kBlock / 64][kRing];
    __shared__ uint32_t s_raux[kBlock / 64][kRing];
    extern __shared__ uint32_t s_reg32[];
    uint8_t *s_reg = reinterpret_cast<uint8_t *>(s_reg32);
    card_begin(c, s_reg32);
    const int wv = threadIdx.x >> 6;
    OccRing ring{s_rkey[wv], s_raux[wv], 0u, 0u};
    OccCursor cur{0ull, kOccChunk};
    uint32_t npos = 0;
    auto flush = [&](uint32_t n) {
        uint4 kk = make_uint4(0, 0, 0, 0);
        uint32_t e = 0;
        ring_take(ring, n, kk, e);
        occ_emit(out, cur, n, kk, (uint8_t)e);
    };
    var_windows<false>(a, n_tiles, s_off, s_pre, [&](bool act, const Occ &o, int64_t j) {
        card_window<KW>(c, s_reg, act, o, j, npos);
        ring_push(ring, act, o.hi, o.lo, (uint32_t)(o.left | (o.right << 4)));
        if (ring.tail - ring.head >= 64) flush(64);
    });
    if (ring.tail != ring.head) flush(ring.tail - ring.head);
    card_end(c, s_reg, npos);
    occ_close(out, cur);
}

// Distinct-sample size and kept count; heavy hitters of the window sample.
template <int KW>
__global__ __launch_bounds__(kBlock) void k_card_tables(const Slot *ss, uint64_t scap, const Slot *hs, uint64_t hcap,
                                                        uint32_t min_depth, uint32_t heavy_min, uint64_t *heavy_keys,
                                                        uint64_t heavy_cap, hm_card_summary_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t nd = 0, nk = 0;
    uint32_t tl[4], tr[4];
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < scap; i += stride) {
        const Slot *s = ss + i;
        if (s->a == 0) continue;
        const uint64_t cnt = slot_counts(s, tl, tr);
        ++nd;
        nk += cnt >= min_depth ? 1u : 0u;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < hcap; i += stride) {
        const Slot *s = hs + i;
        if (s->a == 0) continue;
        if (slot_counts(s, tl, tr) < heavy_min) continue;
        const unsigned long long idx = atomicAdd(reinterpret_cast<unsigned long long *>(&out->n_heavy), 1ull);
        if (idx < heavy_cap) {
            uint64_t hi = 0, lo;
            if (KW == 1) {
                lo = s->a & kLow63;
            } else {
                const uint64_t A = s->a & kLow63, B = s->b & kLow63;
                lo = B | (A << 63);
                hi = A >> 1;
            }
            heavy_keys[2 * idx] = hi;
            heavy_keys[2 * idx + 1] = lo;
        }
    }
    uint64_t d = nd, kk = nk;
    for (int off = 32; off > 0; off >>= 1) {
        d += __shfl_xor(d, off);
        kk += __shfl_xor(kk, off);
    }
    if (lane_id() == 0) {
        if (d) atomicAdd(reinterpret_cast<unsigned long long *>(&out->sampled_distinct), (unsigned long long)d);
        if (kk) atomicAdd(reinterpret_cast<unsigned long long *>(&out->sampled_kept), (unsigned long long)kk);
    }
}

// HyperLogLog estimate from the registers (one workgroup): a histogram of
// register values, then alpha_m m^2 / sum 2^-M[j] with the small-range
// (linear counting) correction of Flajolet et al.
__global__ __launch_bounds__(kBlock) void k_card_estimate(const uint32_t *regs, int p,
                                                          const unsigned long long *positions,
                                                          hm_card_summary_t *out) {
    __shared__ uint32_t hist[66];
    for (int i = threadIdx.x; i < 66; i += kBlock) hist[i] = 0;
    __syncthreads();
    const uint32_t m = 1u << p;
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) atomicAdd(&hist[min(regs[i], 65u)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int r = 0; r <= 65; ++r) sum += (double)hist[r] * ldexp(1.0, -r);
        const double md = (double)m;
        const double alpha = m == 16 ? 0.673 : m == 32 ? 0.697 : m == 64 ? 0.709 : 0.7213 / (1.0 + 1.079 / md);
        double e = alpha * md * md / sum;
        if (e <= 2.5 * md && hist[0] > 0) e = md * log(md / (double)hist[0]);
        out->estimate = e;
        out->positions = *positions;
    }
}

int check_card(const hm_card_t *c) {
    if (!c || !c->registers || !c->positions) return fail(HM_EINVAL, "cardinality: sketch or its buffers are NULL");
    if (c->hll_p < 4 || c->hll_p > kCardMaxP) return fail(HM_EINVAL, "cardinality: hll_p must be 4..%d", kCardMaxP);
    if (c->sample_log2 > 63 || c->heavy_log2 > 63) return fail(HM_EINVAL, "cardinality: sample bits must be 0..63");
    int rc = check_table(&c->sample);
    if (rc) return rc;
    return check_table(&c->heavy);
}

uint32_t probe_bound(const hm_table_t &t) {
    const uint64_t mp = t.max_probe ? (uint64_t)t.max_probe : (uint64_t)kDefaultMaxProbe;
    return (uint32_t)(mp < t.capacity ? mp : t.capacity);
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

int hm_card_init(hm_card_t *c, hipStream_t s) {
    int rc = check_card(c);
    if (rc) return rc;
    rc = fill<uint32_t>(c->registers, 1ull << c->hll_p, 0u, s);
    if (rc) return rc;
    rc = fill<uint64_t>(c->positions, 1, 0ull, s);
    if (rc) return rc;
    rc = hm_table_init(&c->sample, s);
    if (rc) return rc;
    return hm_table_init(&c->heavy, s);
}

// Checks and kernel arguments shared by hm_cardinality and hm_cardinality_occ.
static int card_setup(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, PassArgs &a, CardArgs &ca) {
    int rc = hm_check_params(p);
    if (rc) return rc;
    rc = check_card(c);
    if (rc) return rc;
    if (c->sample.k != p->k || c->heavy.k != p->k)
        return fail(HM_EINVAL, "cardinality: sample tables built for k=%d/%d, params have k=%d", c->sample.k,
                    c->heavy.k, p->k);
    rc = check_reads(r, p->k);
    if (rc) return rc;
    memset(&a, 0, sizeof a);
    a.b2 = r->bases2;
    a.nm = r->nmask;
    a.hq = r->hqmask;
    a.read_off = r->read_off;
    a.n_reads = r->n_reads;
    a.n_bases = r->n_bases;
    a.read_len = r->read_len;
    a.k = p->k;
    a.forward_only = (p->flags & HM_FORWARD_ONLY) ? 1 : 0;
    a.n_owners = p->n_owners;
    a.owner = p->owner;
    a.status = c->sample.status;
    ca.regs = c->registers;
    ca.p = c->hll_p;
    ca.smask = c->sample_log2 ? (~0ull >> (64 - c->sample_log2)) : 0ull;
    ca.hmask = c->heavy_log2 ? (~0ull >> (64 - c->heavy_log2)) : 0ull;
    ca.s_slots = reinterpret_cast<Slot *>(c->sample.slots);
    ca.s_cmask = c->sample.capacity - 1;
    ca.s_probe = probe_bound(c->sample);
    ca.s_status = c->sample.status;
    ca.h_slots = reinterpret_cast<Slot *>(c->heavy.slots);
    ca.h_cmask = c->heavy.capacity - 1;
    ca.h_probe = probe_bound(c->heavy);
    ca.h_status = c->heavy.status;
    ca.positions = reinterpret_cast<unsigned long long *>(c->positions);
    ca.seed = p->seed;
    return HM_OK;
}

// Launch the pass over the reads; `out` NULL: no occurrence stream.
static int card_launch(const hm_reads_t *r, const hm_params_t *p, const hm_card_t *c, const PassArgs &a,
                       const CardArgs &ca, const OccOut *out, hipStream_t s) {
    const bool two = p->k >= 32;
    const size_t lds = (size_t)1 << c->hll_p;
    const int grid_cap = device_cus() * kCardBlocksPerCu;
    if (!r->read_off && r->read_len <= kTileBases - 64) {
        if (r->read_len < p->k) return HM_OK;
        const int32_t rpt = kTileBases / r->read_len;
        const int64_t n_tiles = (r->n_reads + rpt - 1) / rpt;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
        if (out) {
            if (two) hipLaunchKernelGGL(k_card_fixed_occ<2>, g, dim3(kBlock), lds, s, a, ca, *out, rpt, n_tiles);
            else hipLaunchKernelGGL(k_card_fixed_occ<1>, g, dim3(kBlock), lds, s, a, ca, *out, rpt, n_tiles);
        } else {
            const BinHist none{nullptr, 0, 0};
            if (two) hipLaunchKernelGGL((k_card_fixed<2, false>), g, dim3(kBlock), lds, s, a, ca, rpt, n_tiles, none);
            else hipLaunchKernelGGL((k_card_fixed<1, false>), g, dim3(kBlock), lds, s, a, ca, rpt, n_tiles, none);
        }
    } else {
        if (!r->read_off) return fail(HM_EINVAL, "reads longer than %d bases need read_off", kTileBases - 64);
        const int64_t n_tiles = (r->n_reads + kVarReads - 1) / kVarReads;
        const dim3 g((unsigned)(n_tiles < grid_cap ? n_tiles : grid_cap));
        if (out) {
            if (two) hipLaunchKernelGGL(k_card_var_occ<2>, g, dim3(kBlock), lds, s, a, ca, *out, n_tiles);
            else hipLaunchKernelGGL(k_card_var_occ<1>, g, dim3(kBlock), lds, s, a, ca, *out, n_tiles);
        } else {
            if (two) hipLaunchKernelGGL(k_card_var<2>, g, dim3(kBlock), lds, s, a, ca, n_tiles);
            else hipLaunchKernelGGL(k_card_var<1>, g, dim3(kBlock), lds, s, a, ca, n_tiles);
        }
    }
    HM_LAUNCH_CHECK(out ? "hm_cardinality_occ" : "hm_cardinality");
    return HM_OK;
}

int hm_cardinality(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hipStream_t s) {
    PassArgs a;
    CardArgs ca;
    int rc = card_setup(r, p, c, a, ca);
    if (rc) return rc;
    if (r->n_reads == 0) return HM_OK;
    return card_launch(r, p, c, a, ca, nullptr, s);
}

int hm_cardinality_bins(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hm_bins_t *b, hipStream_t s) {
    PassArgs a;
    CardArgs ca;
    int rc = card_setup(r, p, c, a, ca);
    if (rc) return rc;
    rc = check_bins(b);
    if (rc) return rc;
    if (r->read_off || r->read_len > kTileBases - 64)
        return fail(HM_EINVAL, "hm_cardinality_bins needs fixed-length reads of at most %d bases", kTileBases - 64);
    const int32_t rpt = r->read_len > 0 ? kTileBases / r->read_len : 1;
    const int64_t n_tiles = (r->n_reads + rpt - 1) / rpt;
    const int g1 = bins_grid1(n_tiles, b->group_bits);  // the tiles of each workgroup are those hm_bin_kmers scatters
    const int ng = 1 << b->group_bits;
    const size_t lds = ((size_t)1 << c->hll_p) + 4 * (size_t)ng;
    if (lds > 65536)
        return fail(HM_EINVAL, "hm_cardinality_bins: 2^hll_p register bytes and 4 bytes per group exceed 64 KiB "
                    "(hll_p %d, %d groups)", c->hll_p, ng);
    if (r->n_reads == 0 || r->read_len < p->k) {  // no windows: the partition needs no histogram
        bins_note_counted(b, r, p);
        return HM_OK;
    }
    const BinHist bh{bins_hist1(b), (int)(b->group_bits + b->bin_bits), (int)b->bin_bits};
    // the partition's grid is small (a few workgroups a CU): larger workgroups keep the CUs busy
    if (p->k >= 32)
        hipLaunchKernelGGL((k_card_fixed<2, true, kCardHistBlock>), dim3(g1), dim3(kCardHistBlock), lds, s, a, ca, rpt,
                           n_tiles, bh);
    else
        hipLaunchKernelGGL((k_card_fixed<1, true, kCardHistBlock>), dim3(g1), dim3(kCardHistBlock), lds, s, a, ca, rpt,
                           n_tiles, bh);
    HM_LAUNCH_CHECK("hm_cardinality_bins");
    bins_note_counted(b, r, p);
    return HM_OK;
}

int hm_cardinality_occ(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hm_occ_t *o, hipStream_t s) {
    PassArgs a;
    CardArgs ca;
    int rc = card_setup(r, p, c, a, ca);
    if (rc) return rc;
    rc = check_occ(o);
    if (rc) return rc;
    if (r->n_reads == 0) return HM_OK;
    const OccOut out{o->keys, o->ext, o->capacity, reinterpret_cast<unsigned long long *>(o->count)};
    return card_launch(r, p, c, a, ca, &out, s);
}

int hm_card_summary(const hm_card_t *c, uint32_t min_depth, uint32_t heavy_min, uint64_t *heavy_keys,
                    uint64_t heavy_cap, hm_card_summary_t *out, hipStream_t s) {
    int rc = check_card(c);
    if (rc) return rc;
    if (!out) return fail(HM_EINVAL, "cardinality summary: out is NULL");
    if (heavy_cap > 0 && !heavy_keys) return fail(HM_EINVAL, "cardinality summary: heavy_keys is NULL");
    if (c->sample.k != c->heavy.k || c->sample.k < 1 || c->sample.k > 63)
        return fail(HM_EINVAL, "cardinality summary: sample tables disagree on k");
    static_assert(sizeof(hm_card_summary_t) == 40, "summary layout");
    rc = fill<uint64_t>(reinterpret_cast<uint64_t *>(out), sizeof(hm_card_summary_t) / 8, 0ull, s);
    if (rc) return rc;
    const uint64_t cap = c->sample.capacity > c->heavy.capacity ? c->sample.capacity : c->heavy.capacity;
    const dim3 g((unsigned)grid_for(cap, 16));
    const Slot *ss = reinterpret_cast<const Slot *>(c->sample.slots);
    const Slot *hs = reinterpret_cast<const Slot *>(c->heavy.slots);
    if (c->sample.k >= 32)
        hipLaunchKernelGGL(k_card_tables<2>, g, dim3(kBlock), 0, s, ss, c->sample.capacity, hs, c->heavy.capacity,
                           min_depth, heavy_min, heavy_keys, heavy_cap, out);
    else
        hipLaunchKernelGGL(k_card_tables<1>, g, dim3(kBlock), 0, s, ss, c->sample.capacity, hs, c->heavy.capacity,
                           min_depth, heavy_min, heavy_keys, heavy_cap, out);
    HM_LAUNCH_CHECK("hm_card_summary (tables)");
    hipLaunchKernelGGL(k_card_estimate, dim3(1), dim3(kBlock), 0, s, c->registers, c->hll_p,
                       reinterpret_cast<const unsigned long long *>(c->positions), out);
    HM_LAUNCH_CHECK("hm_card_summary (estimate)");
    return HM_OK;
}

}  // extern "C"
