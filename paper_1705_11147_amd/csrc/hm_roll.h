// Windows of fixed-length reads taken a run at a time: a lane extracts the first window of a run
// of kCardRun consecutive windows of one read (forward code and reverse complement) from the
// packed words, and rolls each next window in from one more base: the forward code shifts left
// and appends the base, the reverse complement shifts right and inserts the complemented base on
// top.  Shared by the cardinality pass and the binned partition, which must see the same keys.
#pragma once

#include "hm_device.h"

namespace hm {

constexpr int kCardRun = 8;

// What a run of kCardRun windows starting at base j0 (relative to the tile
// origin) reads besides its first window, in registers: the invalid-base bits
// from j0 on (128 bits, first base most significant), which cover every
// window of the run since kCardRun - 1 + k <= 70, and the 7 bases the run
// rolls in (j0 + k .. j0 + k + 6).  Two loads of mask words and two of base
// words per run instead of an LDS round trip per window.
struct RunBits {
    uint64_t m0, m1;  // invalid-base bits of bases j0 .. j0 + 127
    uint64_t in;      // bases j0 + k .. j0 + k + 31, first base most significant
    __device__ __forceinline__ void load(const Words &w, int64_t j0, int k) {
        const int64_t i = j0 >> 6;
        const int s = (int)(j0 & 63);
        const uint64_t a = w.nm[i], b = w.nm[i + 1], c = w.nm[i + 2];
        m0 = s ? (a << s) | (b >> (64 - s)) : a;
        m1 = s ? (b << s) | (c >> (64 - s)) : b;
        const int64_t p = 2 * (j0 + k);
        const int64_t q = p >> 6;
        const int t = (int)(p & 63);
        const uint64_t x = w.b2[q], y = w.b2[q + 1];
        in = t ? (x << t) | (y >> (64 - t)) : x;
    }
    // window j0 + i (0 <= i < kCardRun) holds no invalid base
    __device__ __forceinline__ bool valid(int i, int k) const {
        const uint64_t m = i ? (m0 << i) | (m1 >> (64 - i)) : m0;
        return (m >> (64 - k)) == 0;
    }
    // bit i (i < cnt) set: window j0 + i holds no invalid base.  One test covers the run's
    // k + kCardRun - 1 bases; only a run that holds an invalid base tests its windows one by one.
    __device__ __forceinline__ uint32_t valid_mask(int k, int cnt) const {
        const uint32_t live = (1u << cnt) - 1u;
        const int span = k + kCardRun - 1;  // <= 70
        const bool clean = span <= 64 ? (m0 >> (64 - span)) == 0 : (m0 == 0 && (m1 >> (128 - span)) == 0);
        if (clean) return live;
        uint32_t v = 0;
        for (int i = 0; i < kCardRun; ++i) v |= valid(i, k) ? 1u << i : 0u;
        return v & live;
    }
    // the base window j0 + i (1 <= i < kCardRun) rolls in: base j0 + i + k - 1
    __device__ __forceinline__ uint64_t base(int i) const { return (in >> (64 - 2 * i)) & 3; }
};

// The forward code and the reverse complement of a window in 2 * KW words of 32 bits (word 0
// least significant), moved on by one base with funnel shifts: the forward code shifts left and
// takes the base at the bottom, the reverse complement shifts right and takes the complemented
// base at bit 2k - 2.  The masks and the word and shift of bit 2k - 2 are the same for every
// lane (set once per launch).
template <int KW>
struct Roll {
    static constexpr int N = 2 * KW;
    uint32_t f[N], r[N];
    struct Shape {
        uint32_t m_top, m_next;  // masks of the two top words of the forward code
        int ts;                  // bit 2k - 2 within the two top words (it always lies there)
    };
    __device__ static Shape shape(int k) {
        const int kb = 2 * k;
        Shape s;
        const int lo_bits = kb - 32 * (N - 2);  // bits in the two top words (KW = 1: the only two)
        s.m_next = lo_bits >= 32 ? ~0u : (1u << lo_bits) - 1u;
        s.m_top = lo_bits > 32 ? (lo_bits >= 64 ? ~0u : (1u << (lo_bits - 32)) - 1u) : 0u;
        s.ts = kb - 2 - 32 * (N - 2);
        return s;
    }
    __device__ __forceinline__ void set(U128 x, U128 y) {
        f[0] = (uint32_t)x.lo, f[1] = (uint32_t)(x.lo >> 32);
        r[0] = (uint32_t)y.lo, r[1] = (uint32_t)(y.lo >> 32);
        if (KW == 2) {
            f[2] = (uint32_t)x.hi, f[3] = (uint32_t)(x.hi >> 32);
            r[2] = (uint32_t)y.hi, r[3] = (uint32_t)(y.hi >> 32);
        }
    }
    __device__ __forceinline__ void step(uint32_t b, const Shape &s) {
#pragma unroll
        for (int i = N - 1; i > 0; --i) f[i] = __builtin_amdgcn_alignbit(f[i], f[i - 1], 30);
        f[0] = (f[0] << 2) | b;
        f[N - 1] &= s.m_top;
        f[N - 2] &= s.m_next;
#pragma unroll
        for (int i = 0; i < N - 1; ++i) r[i] = __builtin_amdgcn_alignbit(r[i + 1], r[i], 2);
        r[N - 1] >>= 2;
        const uint64_t c = (uint64_t)(b ^ 3u) << s.ts;
        r[N - 2] |= (uint32_t)c;
        r[N - 1] |= (uint32_t)(c >> 32);
    }
    __device__ __forceinline__ uint64_t fhi() const { return KW == 2 ? ((uint64_t)f[3] << 32) | f[2] : 0; }
    __device__ __forceinline__ uint64_t flo() const { return ((uint64_t)f[1] << 32) | f[0]; }
    __device__ __forceinline__ uint64_t rhi() const { return KW == 2 ? ((uint64_t)r[3] << 32) | r[2] : 0; }
    __device__ __forceinline__ uint64_t rlo() const { return ((uint64_t)r[1] << 32) | r[0]; }
    // the forward code is the canonical key (it is not larger than the reverse complement)
    __device__ __forceinline__ bool forward() const {
        const uint64_t a = fhi(), c = rhi();
        return a < c || (a == c && flo() <= rlo());
    }
};

// The extensions of a run's windows, in registers: the bases before them (j0 - 1 .. j0 + 30) and
// the high-quality bits around them (from j0 - 1 and from j0 + k), first base most significant.
// The bases after them (j0 + k ..) are RunBits::in.  At the tile origin (j0 = 0) the base and bit
// before it read as 0; no read starts before the origin, so no window uses them.
struct RunExt {
    uint64_t pre;       // bases j0 - 1 .. j0 + 30
    uint64_t hql, hqr;  // high-quality bits of bases j0 - 1 .. j0 + 62 and j0 + k .. j0 + k + 63
    __device__ static uint64_t bits_at(const uint64_t *m, int64_t j) {  // 64 bits from bit j
        const int64_t i = j >> 6;
        const int s = (int)(j & 63);
        return s ? (m[i] << s) | (m[i + 1] >> (64 - s)) : m[i];
    }
    __device__ __forceinline__ void load(const Words &w, int64_t j0, int k) {
        if (j0 > 0) {
            pre = bits_at(w.b2, 2 * (j0 - 1));
            hql = bits_at(w.hq, j0 - 1);
        } else {
            pre = w.b2[0] >> 2;
            hql = w.hq[0] >> 1;
        }
        hqr = bits_at(w.hq, j0 + k);
    }
    // the extensions of window j0 + i of a read spanning [rb, re): left and right base (4 = none),
    // forward strand
    __device__ __forceinline__ void fwd_ext(const RunBits &r, int i, int64_t j0, int64_t rb, int64_t re, int k,
                                            int &left, int &right) const {
        const int64_t j = j0 + i;
        const bool lok = j > rb && ((hql >> (63 - i)) & 1);
        const bool rok = j + k < re && ((hqr >> (63 - i)) & 1);
        left = lok ? (int)((pre >> (62 - 2 * i)) & 3) : 4;
        right = rok ? (int)((r.in >> (62 - 2 * i)) & 3) : 4;
    }
};

}  // namespace hm
