/*
 * Seeded synthetic genomes and reads for the k-mer analysis workloads.
 *
 * This file only simulates sequencing data: uniform random genomes, repeat
 * copies with divergence, homeologous copies, and reads with substitution
 * errors and Phred qualities.  It contains none of the k-mer analysis
 * arithmetic (no encoding, canonical form, hashing or counting), so both the
 * CPU oracle and the GPU path can consume its output without sharing code.
 *
 * Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) run as a counter-based
 * generator.  Every read and every genome chunk seeds its own stream from
 * (seed, stream tag, index), so the output does not depend on the number of
 * OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t x; } rng_t;

static inline void rng_init(rng_t *r, uint64_t seed, uint64_t tag, uint64_t idx) {
    r->x = sm_mix(seed ^ sm_mix(tag * GOLDEN + 0x5851F42D4C957F2DULL) ^ sm_mix(idx + 0x14057B7EF767814FULL));
}
static inline uint64_t rng_u64(rng_t *r) {
    r->x += GOLDEN;
    return sm_mix(r->x);
}
/* uniform in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_u64(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, n) by multiply-high (Lemire) */
static inline uint64_t rng_below(rng_t *r, uint64_t n) {
    return (uint64_t)(((unsigned __int128)rng_u64(r) * n) >> 64);
}

static const uint8_t ACGT[4] = {'A', 'C', 'G', 'T'};

static inline uint8_t comp_ascii(uint8_t b) {
    switch (b) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 'N';
    }
}

/* index of an uppercase base in ACGT, for picking a different base */
static inline int base_idx(uint8_t b) {
    switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    default: return 3;
    }
}

/* a uniformly chosen base different from b */
static inline uint8_t substitute(rng_t *r, uint8_t b) {
    int i = base_idx(b);
    int j = (int)rng_below(r, 3);
    return ACGT[j >= i ? j + 1 : j];
}

#define CHUNK 65536

/* Uniform ACGT genome of n bases. */
void syn_genome_uniform(uint8_t *out, int64_t n, uint64_t seed) {
    int64_t nchunk = (n + CHUNK - 1) / CHUNK;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunk; ++c) {
        rng_t r;
        rng_init(&r, seed, 1, (uint64_t)c);
        int64_t b = c * CHUNK, e = b + CHUNK < n ? b + CHUNK : n;
        int64_t i = b;
        while (i < e) {
            uint64_t x = rng_u64(&r);
            for (int j = 0; j < 32 && i < e; ++j, ++i) out[i] = ACGT[(x >> (2 * j)) & 3];
        }
    }
}

/* Copy src[0..n) to dst with iid substitutions at rate div (each chosen
 * position gets a uniformly chosen different base). */
void syn_diverge(const uint8_t *src, uint8_t *dst, int64_t n, double div, uint64_t seed, uint64_t tag) {
    int64_t nchunk = (n + CHUNK - 1) / CHUNK;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunk; ++c) {
        rng_t r;
        rng_init(&r, seed, 2 + tag * 16, (uint64_t)c);
        int64_t b = c * CHUNK, e = b + CHUNK < n ? b + CHUNK : n;
        for (int64_t i = b; i < e; ++i) {
            uint8_t x = src[i];
            dst[i] = rng_unif(&r) < div ? substitute(&r, x) : x;
        }
    }
}

/* Segmental repeats (the mid-size workload): copy segments of length
 * U[min_len, max_len] taken from random positions of the genome, diverge
 * each copy by `div`, and overwrite random positions until `target` bases
 * have been written.  Sequential, so the result is deterministic. */
int64_t syn_segmental_repeats(uint8_t *g, int64_t G, int64_t min_len, int64_t max_len, double div,
                              int64_t target, uint64_t seed) {
    rng_t r;
    rng_init(&r, seed, 3, 0);
    uint8_t *buf = (uint8_t *)malloc((size_t)max_len);
    if (!buf) return -1;
    int64_t written = 0, copies = 0;
    while (written < target) {
        int64_t len = min_len + (int64_t)rng_below(&r, (uint64_t)(max_len - min_len + 1));
        if (len > G) len = G;
        int64_t src = (int64_t)rng_below(&r, (uint64_t)(G - len + 1));
        int64_t dst = (int64_t)rng_below(&r, (uint64_t)(G - len + 1));
        for (int64_t i = 0; i < len; ++i) {
            uint8_t x = g[src + i];
            buf[i] = rng_unif(&r) < div ? substitute(&r, x) : x;
        }
        memcpy(g + dst, buf, (size_t)len);
        written += len;
        ++copies;
    }
    free(buf);
    return copies;
}

/* Interspersed repeat families (the human-scale workload): n_fam consensus
 * sequences of log-uniform length in [min_len, max_len]; each copy takes a
 * random family and a divergence ~ U(div_lo, div_hi) from its consensus, and
 * overwrites a uniform position, until `target` bases have been written. */
int64_t syn_interspersed_repeats(uint8_t *g, int64_t G, int32_t n_fam, int64_t min_len, int64_t max_len,
                                 double div_lo, double div_hi, int64_t target, uint64_t seed) {
    rng_t r;
    rng_init(&r, seed, 4, 0);
    int64_t *flen = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_fam);
    int64_t *foff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_fam + 1));
    if (!flen || !foff) return -1;
    double lmin = log((double)min_len), lmax = log((double)max_len);
    foff[0] = 0;
    for (int32_t f = 0; f < n_fam; ++f) {
        flen[f] = (int64_t)llround(exp(lmin + (lmax - lmin) * rng_unif(&r)));
        foff[f + 1] = foff[f] + flen[f];
    }
    uint8_t *cons = (uint8_t *)malloc((size_t)foff[n_fam]);
    if (!cons) return -1;
    for (int64_t i = 0; i < foff[n_fam]; ++i) cons[i] = ACGT[rng_below(&r, 4)];
    int64_t written = 0, copies = 0;
    while (written < target) {
        int32_t f = (int32_t)rng_below(&r, (uint64_t)n_fam);
        int64_t len = flen[f] < G ? flen[f] : G;
        double div = div_lo + (div_hi - div_lo) * rng_unif(&r);
        int64_t dst = (int64_t)rng_below(&r, (uint64_t)(G - len + 1));
        const uint8_t *c = cons + foff[f];
        for (int64_t i = 0; i < len; ++i) g[dst + i] = rng_unif(&r) < div ? substitute(&r, c[i]) : c[i];
        written += len;
        ++copies;
    }
    free(cons);
    free(foff);
    free(flen);
    return copies;
}

/* CDF of clamp(rint(N(mu, sd)), qmin, qmax) over q = 0..63, scaled to 2^53. */
static void phred_cdf(double mu, double sd, int qmin, int qmax, uint64_t cdf[64]) {
    for (int q = 0; q < 64; ++q) {
        double p;
        if (q < qmin) p = 0.0;
        else if (q >= qmax) p = 1.0;
        else p = 0.5 * erfc(-((q + 0.5) - mu) / (sd * sqrt(2.0)));
        cdf[q] = (uint64_t)(p * 9007199254740992.0);
    }
    cdf[63] = 9007199254740992ULL;
}

/*
 * Sample reads [r0, r0 + n) of a read set.
 *   genome / chrom_off[n_chrom + 1]: chromosomes concatenated; reads never
 *     cross a chromosome boundary; start uniform over all valid starts.
 *   L: read length.  Half the reads (probability 1/2) are reverse complemented.
 *   err_mean: mean substitution rate.  end_bias != 0 makes the per-position
 *     rate proportional to 1 + 2 * |2i/(L-1) - 1|^2 (read ends 3x the
 *     centre), scaled so its mean over the read is err_mean.
 *   Phred: iid clamp(rint(N(q_mu, q_sd)), q_min, q_max), independent of the
 *     errors, written as numeric bytes (no ASCII offset).
 * Outputs ascii[n * L], qual[n * L]; optional start/strand arrays (may be NULL).
 */
int syn_reads(const uint8_t *genome, const int64_t *chrom_off, int32_t n_chrom, int32_t L, int64_t r0, int64_t n,
              uint64_t seed, double err_mean, int32_t end_bias, double q_mu, double q_sd, int32_t q_min,
              int32_t q_max, uint8_t *ascii, uint8_t *qual, int64_t *start_out, uint8_t *strand_out) {
    if (L <= 0 || n_chrom <= 0) return -1;
    int64_t *cum = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_chrom + 1));
    if (!cum) return -1;
    cum[0] = 0;
    for (int32_t c = 0; c < n_chrom; ++c) {
        int64_t len = chrom_off[c + 1] - chrom_off[c];
        cum[c + 1] = cum[c] + (len >= L ? len - L + 1 : 0);
    }
    if (cum[n_chrom] <= 0) {
        free(cum);
        return -2;
    }
    double *perr = (double *)malloc(sizeof(double) * (size_t)L);
    if (!perr) {
        free(cum);
        return -1;
    }
    double wsum = 0.0;
    for (int i = 0; i < L; ++i) {
        double w = 1.0;
        if (end_bias && L > 1) {
            double t = fabs(2.0 * i / (double)(L - 1) - 1.0);
            w = 1.0 + 2.0 * t * t;
        }
        perr[i] = w;
        wsum += w;
    }
    for (int i = 0; i < L; ++i) perr[i] = err_mean * perr[i] * L / wsum;
    uint64_t cdf[64];
    phred_cdf(q_mu, q_sd, q_min, q_max, cdf);
    /* guide table: guide[t] = smallest q whose cdf exceeds t / 4096 of the range */
    uint8_t guide[4096];
    for (int t = 0, qq = 0; t < 4096; ++t) {
        uint64_t lo_u = (uint64_t)t << 41;
        while (qq < 63 && cdf[qq] <= lo_u) ++qq;
        guide[t] = (uint8_t)qq;
    }
    int64_t total = cum[n_chrom];

#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        int64_t rid = r0 + j;
        rng_t r;
        rng_init(&r, seed, 5, (uint64_t)rid);
        int64_t v = (int64_t)rng_below(&r, (uint64_t)total);
        int32_t lo = 0, hi = n_chrom; /* find c with cum[c] <= v < cum[c+1] */
        while (hi - lo > 1) {
            int32_t mid = (lo + hi) / 2;
            if (cum[mid] <= v) lo = mid;
            else hi = mid;
        }
        int64_t start = chrom_off[lo] + (v - cum[lo]);
        int strand = (int)(rng_u64(&r) & 1);
        uint8_t *a = ascii + j * (int64_t)L;
        uint8_t *q = qual + j * (int64_t)L;
        const uint8_t *s = genome + start;
        if (!strand) {
            memcpy(a, s, (size_t)L);
        } else {
            for (int i = 0; i < L; ++i) a[i] = comp_ascii(s[L - 1 - i]);
        }
        for (int i = 0; i < L; ++i) {
            if (rng_unif(&r) < perr[i]) a[i] = substitute(&r, a[i]);
        }
        for (int i = 0; i < L; ++i) {
            uint64_t u = rng_u64(&r) >> 11;
            int qq = guide[u >> 41];
            while (qq < 63 && u >= cdf[qq]) ++qq;
            q[i] = (uint8_t)qq;
        }
        if (start_out) start_out[j] = start;
        if (strand_out) strand_out[j] = (uint8_t)strand;
    }
    free(perr);
    free(cum);
    return 0;
}
