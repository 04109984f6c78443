/*
 * TEST INFRASTRUCTURE -- CPU oracle for HipMer k-mer analysis.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU path: no headers,
 * helpers, tables or constants.  It computes the plain definition of k-mer
 * analysis with a std::unordered_map and std::sort; there is no Bloom filter,
 * because the Bloom pass only removes singletons, which the depth filter
 * removes anyway (k-mer analysis, section "Parallel k-mer analysis").
 *
 * What is computed (paper section "The Meraculous Assembly Pipeline", step
 * 1, and section "Parallel k-mer analysis"):
 *   - every read is chopped into its overlapping length-k windows (k-mers);
 *   - each distinct k-mer is counted; k-mers seen fewer than min_depth times
 *     are dropped as errors (the epsilon cutoff);
 *   - for every k-mer, two arrays of four counters tally the bases seen
 *     immediately to its left and right in the reads (the "extensions");
 *     a base on a side is a high-quality extension when its tally reaches
 *     ext_min (the t_hq threshold);
 *   - each side is classified as unique (one high-quality base), fork (two
 *     or more) or none (X), and k-mers unique on both sides (UU) are the
 *     ones the de Bruijn graph is built from (section "Parallel contig
 *     generation").
 * Readings where the paper is silent (all listed in the design notes):
 *   - encoding: A=0, C=1, G=2, T=3, first base most significant, so numeric
 *     order is lexicographic order;
 *   - canonical form: the smaller of the k-mer and its reverse complement
 *     (k odd, so they never tie); when the reverse complement is the key,
 *     the two sides swap and their bases are complemented;
 *   - an extension base is tallied only when its Phred quality is >= qcut;
 *     qualities of the bases inside the k-mer are not used;
 *   - a window containing a non-ACGT byte yields no k-mer; a neighbour that
 *     is non-ACGT or beyond the read end yields no tally;
 *   - owner map (owner-computes, section "Parallel k-mer analysis", which
 *     hashes each k-mer to its owner without fixing the function):
 *     own(key) = floor(H(key) * n_owners / 2^64) with
 *     H = (lo ^ hi * 0x9E3779B97F4A7C15) * 0xD1B54A32D192ED03 mod 2^64, the
 *     multiply-shift scheme (the high bits of a product by an odd constant).
 *
 * Threads, two plain schemes (both exact, each pinned by a test):
 *   - key-partitioned (default): thread t of T keeps the keys whose
 *     separately seeded partition hash is t and scans every read; the union
 *     over threads is the table by the owner-partition identity;
 *   - read-partitioned (ORC_SPLIT_READS): thread t counts reads
 *     [t*N/T, (t+1)*N/T) into its own maps, one per key partition, and the
 *     maps are summed key by key before the depth filter, by additivity of
 *     unfiltered tables (thread q sums partition q).
 *   - sort-counted (ORC_SORT_COUNT): thread t writes one record (key, left,
 *     right) per kept window of reads [t*N/T, (t+1)*N/T) into a list per key
 *     partition; thread q then sorts partition q's records by key and reads
 *     each run of equal keys as one k-mer: its count is the run's length and
 *     its tallies count the run's left and right bases.  The same definition,
 *     with a sort in place of the map (no random access per window).
 * Reads may also come in batches (orc_acc_*): counting batch after batch
 * into the same state is the table of their union, by the same additivity.
 * Output records are sorted by key.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

typedef unsigned __int128 u128;

namespace {

constexpr uint64_t kOwnerMul1 = 0x9E3779B97F4A7C15ULL;  /* method-defined owner map */
constexpr uint64_t kOwnerMul2 = 0xD1B54A32D192ED03ULL;
constexpr uint64_t kShardSeed = 0x13198A2E03707344ULL;  /* test sampling shards */
constexpr uint64_t kThreadSeed = 0xA4093822299F31D0ULL; /* oracle thread partition */
constexpr uint64_t kCardSeed = 0xB7E151628AED2A6AULL;   /* method-defined cardinality hash */
constexpr uint64_t kPosSeed = 0x452821E638D01377ULL;    /* method-defined window sampling hash */

inline uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

inline uint64_t key_hash(uint64_t hi, uint64_t lo, uint64_t seed) { return fmix64(fmix64(hi ^ seed) ^ lo); }

inline uint32_t part_of(uint64_t h, uint32_t n) { return (uint32_t)(((u128)h * n) >> 64); }

/* base code: A/a=0 C/c=1 G/g=2 T/t=3, anything else invalid (4) */
inline int code_of(uint8_t b) {
    switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
    }
}

struct Tally {
    uint32_t cnt = 0;
    uint32_t tl[4] = {0, 0, 0, 0};
    uint32_t tr[4] = {0, 0, 0, 0};
};

struct KeyHash {
    size_t operator()(u128 x) const { return (size_t)key_hash((uint64_t)(x >> 64), (uint64_t)x, 0x9E3779B97F4A7C15ULL); }
};

typedef std::unordered_map<u128, Tally, KeyHash> Map;

}  // namespace

extern "C" {

enum { ORC_FORWARD_ONLY = 1, ORC_KEEP_ALL = 2, ORC_SPLIT_READS = 4, ORC_SORT_COUNT = 8 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EOVERFLOW = -2 };

typedef struct {
    int32_t k;
    int32_t qual_offset;
    int32_t qcut;
    uint32_t min_depth;
    uint32_t ext_min;
    uint32_t n_owners; /* method owner filter; 1 = keep every key */
    uint32_t owner;
    uint32_t n_shards; /* test sampling: keep only keys of shard `shard` */
    uint32_t shard;
    uint32_t flags;
    int32_t n_threads;
} orc_params_t;

struct orc_result {
    std::vector<u128> key;
    std::vector<Tally> val;
    int64_t positions = 0; /* valid k-mer windows scanned (before owner/shard filters) */
};

inline uint64_t owner_hash(uint64_t hi, uint64_t lo) { return (lo ^ hi * kOwnerMul1) * kOwnerMul2; }
uint32_t orc_owner(uint64_t hi, uint64_t lo, uint32_t n_owners) { return part_of(owner_hash(hi, lo), n_owners); }
uint32_t orc_shard(uint64_t hi, uint64_t lo, uint32_t n_shards) { return part_of(key_hash(hi, lo, kShardSeed), n_shards); }

/* vector forms for filtering exported records: which = 0 owner map, 1 shard */
void orc_part_many(const uint64_t *hi, const uint64_t *lo, int64_t n, uint32_t n_parts, int32_t which, uint32_t *out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = which == 0 ? orc_owner(hi[i], lo[i], n_parts) : orc_shard(hi[i], lo[i], n_parts);
}

/* class of one side: the base if exactly one base reaches ext_min, 4 (fork)
 * if several do, 5 (X, no neighbour) if none does */
static uint8_t classify(const uint32_t t[4], uint32_t ext_min) {
    int n = 0, b = -1;
    for (int i = 0; i < 4; ++i)
        if (t[i] >= ext_min) {
            ++n;
            b = i;
        }
    if (n == 0) return 5;
    if (n == 1) return (uint8_t)b;
    return 4;
}

/* Count the windows of reads [0, n_reads) into `maps`.  n_parts > 1: keep
 * only the keys of partition `part` (into maps[0]).  Otherwise, with several
 * maps, file each key under its partition: maps[partition of the key]. */
static int scan_reads(const uint8_t *ascii, const uint8_t *qual, const int64_t *read_off, int64_t n_reads,
                      const orc_params_t *p, uint32_t n_parts, uint32_t part, std::vector<Map> &maps,
                      int64_t *positions) {
    const uint32_t n_file = (uint32_t)maps.size();
    const int k = p->k;
    const u128 mask = (k == 64) ? ~(u128)0 : (((u128)1 << (2 * k)) - 1);
    int64_t npos = 0;
    for (int64_t r = 0; r < n_reads; ++r) {
        const int64_t b = read_off[r];
        const int64_t L = read_off[r + 1] - b;
        const uint8_t *s = ascii + b;
        const uint8_t *q = qual + b;
        /* HQ(j): 0 <= j < L, base valid, Phred >= qcut */
        auto hq = [&](int64_t j) -> bool {
            return j >= 0 && j < L && code_of(s[j]) < 4 && ((int)q[j] - p->qual_offset) >= p->qcut;
        };
        u128 fwd = 0, rc = 0;
        int64_t run = 0; /* length of the current run of valid bases ending at j */
        for (int64_t j = 0; j < L; ++j) {
            const int c = code_of(s[j]);
            if (c == 4) {
                run = 0;
                fwd = rc = 0;
                continue;
            }
            /* enc of the window ending at j, and of its reverse complement */
            fwd = ((fwd << 2) | (u128)c) & mask;
            rc = (rc >> 2) | ((u128)(3 - c) << (2 * (k - 1)));
            if (++run < k) continue;
            ++npos;
            const int64_t i = j - k + 1; /* window start */
            const bool forward_only = (p->flags & ORC_FORWARD_ONLY) != 0;
            const bool is_fwd = forward_only || fwd <= rc;
            const u128 key = is_fwd ? fwd : rc;
            const uint64_t hi = (uint64_t)(key >> 64), lo = (uint64_t)key;
            if (p->n_owners > 1 && orc_owner(hi, lo, p->n_owners) != p->owner) continue;
            if (p->n_shards > 1 && orc_shard(hi, lo, p->n_shards) != p->shard) continue;
            const uint32_t kpart = (n_parts > 1 || n_file > 1)
                                       ? part_of(key_hash(hi, lo, kThreadSeed), n_parts > 1 ? n_parts : n_file) : 0;
            if (n_parts > 1 && kpart != part) continue;
            Map &m = maps[n_parts > 1 ? 0 : kpart];
            int left = -1, right = -1;
            if (is_fwd) {
                if (hq(i - 1)) left = code_of(s[i - 1]);
                if (hq(i + k)) right = code_of(s[i + k]);
            } else {
                if (hq(i + k)) left = 3 - code_of(s[i + k]);
                if (hq(i - 1)) right = 3 - code_of(s[i - 1]);
            }
            Tally &t = m[key];
            if (t.cnt == UINT32_MAX) return ORC_EOVERFLOW;
            ++t.cnt;
            if (left >= 0) ++t.tl[left];
            if (right >= 0) ++t.tr[right];
        }
    }
    *positions = npos;
    return ORC_OK;
}

/* One kept window for the sort-counted scheme: its key and its extension
 * bases (-1: none). */
struct OccRec {
    uint64_t hi, lo;
    int8_t left, right;
};

/* The windows of reads [0, n_reads) as records, each filed under its key
 * partition (recs.size() partitions), with the same filters and extension
 * rule as scan_reads. */
static void scan_records(const uint8_t *ascii, const uint8_t *qual, const int64_t *read_off, int64_t n_reads,
                         const orc_params_t *p, std::vector<std::vector<OccRec>> &recs, int64_t *positions) {
    const uint32_t n_file = (uint32_t)recs.size();
    const int k = p->k;
    const u128 mask = (((u128)1 << (2 * k)) - 1);
    int64_t npos = 0;
    for (int64_t r = 0; r < n_reads; ++r) {
        const int64_t b = read_off[r];
        const int64_t L = read_off[r + 1] - b;
        const uint8_t *s = ascii + b;
        const uint8_t *q = qual + b;
        auto hq = [&](int64_t j) -> bool {
            return j >= 0 && j < L && code_of(s[j]) < 4 && ((int)q[j] - p->qual_offset) >= p->qcut;
        };
        u128 fwd = 0, rc = 0;
        int64_t run = 0;
        for (int64_t j = 0; j < L; ++j) {
            const int c = code_of(s[j]);
            if (c == 4) {
                run = 0;
                fwd = rc = 0;
                continue;
            }
            fwd = ((fwd << 2) | (u128)c) & mask;
            rc = (rc >> 2) | ((u128)(3 - c) << (2 * (k - 1)));
            if (++run < k) continue;
            ++npos;
            const int64_t i = j - k + 1;
            const bool is_fwd = (p->flags & ORC_FORWARD_ONLY) != 0 || fwd <= rc;
            const u128 key = is_fwd ? fwd : rc;
            const uint64_t hi = (uint64_t)(key >> 64), lo = (uint64_t)key;
            if (p->n_owners > 1 && orc_owner(hi, lo, p->n_owners) != p->owner) continue;
            if (p->n_shards > 1 && orc_shard(hi, lo, p->n_shards) != p->shard) continue;
            OccRec o{hi, lo, -1, -1};
            if (is_fwd) {
                if (hq(i - 1)) o.left = (int8_t)code_of(s[i - 1]);
                if (hq(i + k)) o.right = (int8_t)code_of(s[i + k]);
            } else {
                if (hq(i + k)) o.left = (int8_t)(3 - code_of(s[i + k]));
                if (hq(i - 1)) o.right = (int8_t)(3 - code_of(s[i - 1]));
            }
            const uint32_t kpart = n_file > 1 ? part_of(key_hash(hi, lo, kThreadSeed), n_file) : 0;
            recs[kpart].push_back(o);
        }
    }
    *positions = npos;
}

/* The counting state of a run, which may take several read batches (by
 * additivity of unfiltered tables, counting batch after batch into the same
 * maps gives the table of their union).  maps[t][q]: thread t's counts of the
 * keys of partition q (q = 0 only in the key-partitioned scheme, where thread
 * t keeps partition t itself; in the read-partitioned scheme thread t files
 * each key of its reads under its partition, and at the end thread q sums
 * partition q over all threads, so the merge runs in parallel). */
struct orc_acc {
    orc_params_t p;
    uint32_t T;
    bool split;
    bool sorted; /* ORC_SORT_COUNT: recs[t][q] instead of maps */
    std::vector<std::vector<Map>> maps;
    std::vector<std::vector<std::vector<OccRec>>> recs;
    int64_t positions = 0;
};

static void run_threads(uint32_t T, const std::function<void(uint32_t)> &work) {
    if (T == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < T; ++t) th.emplace_back(work, t);
    for (auto &x : th) x.join();
}

/* Count reads [0, n_reads) of one batch into the state. */
static int acc_add(orc_acc *a, const uint8_t *ascii, const uint8_t *qual, const int64_t *read_off, int64_t n_reads) {
    const uint32_t T = a->T;
    std::vector<int> rcs(T, 0);
    std::vector<int64_t> npos(T, 0);
    if (a->sorted) {
        run_threads(T, [&](uint32_t t) {
            const int64_t r0 = n_reads * t / T, r1 = n_reads * (t + 1) / T;
            scan_records(ascii, qual, read_off + r0, r1 - r0, &a->p, a->recs[t], &npos[t]);
        });
        for (auto x : npos) a->positions += x;
        return ORC_OK;
    }
    if (a->split) {
        /* reads [t*N/T, (t+1)*N/T) into thread t's maps, one map per key partition */
        run_threads(T, [&](uint32_t t) {
            const int64_t r0 = n_reads * t / T, r1 = n_reads * (t + 1) / T;
            rcs[t] = scan_reads(ascii, qual, read_off + r0, r1 - r0, &a->p, 1, 0, a->maps[t], &npos[t]);
        });
    } else {
        /* thread t scans every read and keeps the keys of partition t */
        run_threads(T, [&](uint32_t t) {
            rcs[t] = scan_reads(ascii, qual, read_off, n_reads, &a->p, T, t, a->maps[t], &npos[t]);
        });
    }
    for (uint32_t t = 0; t < T; ++t)
        if (rcs[t] != ORC_OK) return rcs[t];
    a->positions += a->split ? [&] { int64_t s = 0; for (auto x : npos) s += x; return s; }() : npos[0];
    return ORC_OK;
}

/* Sum the partitions over threads (read-partitioned scheme), apply the depth
 * filter and sort by key. */
static int64_t acc_finish(orc_acc *a, void **handle) {
    const uint32_t T = a->T;
    std::vector<int> rcs(T, 0);
    if (a->split && T > 1) {
        run_threads(T, [&](uint32_t q) {
            Map &dst = a->maps[0][q];
            for (uint32_t t = 1; t < T; ++t) {
                for (auto &kv : a->maps[t][q]) {
                    Tally &d = dst[kv.first];
                    if ((uint64_t)d.cnt + kv.second.cnt > UINT32_MAX) {
                        rcs[q] = ORC_EOVERFLOW;
                        return;
                    }
                    d.cnt += kv.second.cnt;
                    for (int b = 0; b < 4; ++b) {
                        d.tl[b] += kv.second.tl[b];
                        d.tr[b] += kv.second.tr[b];
                    }
                }
                Map().swap(a->maps[t][q]);
            }
        });
        for (uint32_t q = 0; q < T; ++q)
            if (rcs[q] != ORC_OK) return rcs[q];
    }
    const bool keep_all = (a->p.flags & ORC_KEEP_ALL) != 0;
    std::vector<std::pair<u128, Tally>> recs;
    if (a->sorted) {
        /* thread q: partition q's records from every thread, sorted by key; a run of equal keys is one
           k-mer, counted and tallied over the run */
        std::vector<std::vector<std::pair<u128, Tally>>> out(T);
        run_threads(T, [&](uint32_t q) {
            std::vector<OccRec> v;
            size_t n = 0;
            for (uint32_t t = 0; t < T; ++t) n += a->recs[t][q].size();
            v.reserve(n);
            for (uint32_t t = 0; t < T; ++t) {
                v.insert(v.end(), a->recs[t][q].begin(), a->recs[t][q].end());
                std::vector<OccRec>().swap(a->recs[t][q]);
            }
            std::sort(v.begin(), v.end(), [](const OccRec &x, const OccRec &y) {
                return x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo);
            });
            for (size_t i = 0; i < v.size();) {
                size_t j = i;
                Tally t;
                while (j < v.size() && v[j].hi == v[i].hi && v[j].lo == v[i].lo) {
                    if (v[j].left >= 0) ++t.tl[v[j].left];
                    if (v[j].right >= 0) ++t.tr[v[j].right];
                    ++j;
                }
                if (j - i > UINT32_MAX) {
                    rcs[q] = ORC_EOVERFLOW;
                    return;
                }
                t.cnt = (uint32_t)(j - i);
                if (keep_all || t.cnt >= a->p.min_depth) out[q].push_back({((u128)v[i].hi << 64) | v[i].lo, t});
                i = j;
            }
        });
        for (uint32_t q = 0; q < T; ++q)
            if (rcs[q] != ORC_OK) return rcs[q];
        /* every partition is in key order: merge them (a heap of the partitions' next records) */
        size_t n = 0;
        for (auto &o : out) n += o.size();
        orc_result *res = new orc_result();
        res->positions = a->positions;
        res->key.reserve(n);
        res->val.reserve(n);
        typedef std::pair<u128, uint32_t> Head; /* next key of a partition, the partition */
        std::priority_queue<Head, std::vector<Head>, std::greater<Head>> heap;
        std::vector<size_t> at(T, 0);
        for (uint32_t q = 0; q < T; ++q)
            if (!out[q].empty()) heap.push({out[q][0].first, q});
        while (!heap.empty()) {
            const uint32_t q = heap.top().second;
            heap.pop();
            res->key.push_back(out[q][at[q]].first);
            res->val.push_back(out[q][at[q]].second);
            if (++at[q] < out[q].size()) heap.push({out[q][at[q]].first, q});
        }
        *handle = res;
        return (int64_t)n;
    }
    orc_result *res = new orc_result();
    res->positions = a->positions;
    for (auto &row : a->maps)
        for (auto &m : row) {
            for (auto &kv : m)
                if (keep_all || kv.second.cnt >= a->p.min_depth) recs.push_back(kv);
            Map().swap(m);
        }
    std::sort(recs.begin(), recs.end(), [](const std::pair<u128, Tally> &x, const std::pair<u128, Tally> &y) {
        return x.first < y.first;
    });
    res->key.reserve(recs.size());
    res->val.reserve(recs.size());
    for (auto &kv : recs) {
        res->key.push_back(kv.first);
        res->val.push_back(kv.second);
    }
    *handle = res;
    return (int64_t)recs.size();
}

static int check_params(const orc_params_t *p) {
    if (!p || p->k < 1 || p->k > 63) return ORC_EINVAL;
    if (!(p->flags & ORC_FORWARD_ONLY) && (p->k % 2) == 0) return ORC_EINVAL;
    if (p->n_owners < 1 || p->owner >= p->n_owners) return ORC_EINVAL;
    if (p->n_shards < 1 || p->shard >= p->n_shards) return ORC_EINVAL;
    return ORC_OK;
}

/* A counting state for reads given in several batches (orc_acc_add per
 * batch, then orc_acc_finish); NULL on bad parameters. */
void *orc_acc_new(const orc_params_t *p) {
    if (check_params(p) != ORC_OK) return nullptr;
    orc_acc *a = new orc_acc();
    a->p = *p;
    a->T = p->n_threads > 1 ? (uint32_t)p->n_threads : 1u;
    a->split = (p->flags & ORC_SPLIT_READS) != 0;
    a->sorted = (p->flags & ORC_SORT_COUNT) != 0;
    if (a->sorted) a->recs.assign(a->T, std::vector<std::vector<OccRec>>(a->T));
    else a->maps.assign(a->T, std::vector<Map>(a->split ? a->T : 1));
    return a;
}

int orc_acc_add(void *acc, const uint8_t *ascii, const uint8_t *qual, const int64_t *read_off, int64_t n_reads) {
    if (!acc || n_reads < 0) return ORC_EINVAL;
    return acc_add((orc_acc *)acc, ascii, qual, read_off, n_reads);
}

/* Finish and free the state: records as for orc_run (count or error). */
int64_t orc_acc_finish(void *acc, void **handle) {
    *handle = nullptr;
    if (!acc) return ORC_EINVAL;
    orc_acc *a = (orc_acc *)acc;
    const int64_t n = acc_finish(a, handle);
    delete a;
    return n;
}

void orc_acc_free(void *acc) { delete (orc_acc *)acc; }

/* Run the oracle.  read_off has n_reads + 1 entries (base offsets).  Returns
 * the number of output records (>= 0) or a negative error; *handle receives
 * the result for orc_fetch / orc_free. */
int64_t orc_run(const uint8_t *ascii, const uint8_t *qual, const int64_t *read_off, int64_t n_reads,
                const orc_params_t *p, void **handle) {
    *handle = nullptr;
    if (check_params(p) != ORC_OK || n_reads < 0) return ORC_EINVAL;
    void *a = orc_acc_new(p);
    const int rc = orc_acc_add(a, ascii, qual, read_off, n_reads);
    if (rc != ORC_OK) {
        orc_acc_free(a);
        return rc;
    }
    return orc_acc_finish(a, handle);
}

/* Copy the sorted records out.  tl/tr are n x 4 row-major; cls_* as
 * classify(): 0..3 = unique base A,C,G,T; 4 = fork; 5 = X. */
void orc_fetch(void *handle, uint32_t ext_min, uint64_t *key_hi, uint64_t *key_lo, uint32_t *count, uint32_t *tl,
               uint32_t *tr, uint8_t *cls_l, uint8_t *cls_r) {
    const orc_result *res = (const orc_result *)handle;
    const size_t n = res->key.size();
    for (size_t i = 0; i < n; ++i) {
        key_hi[i] = (uint64_t)(res->key[i] >> 64);
        key_lo[i] = (uint64_t)res->key[i];
        count[i] = res->val[i].cnt;
        for (int b = 0; b < 4; ++b) {
            tl[4 * i + b] = res->val[i].tl[b];
            tr[4 * i + b] = res->val[i].tr[b];
        }
        cls_l[i] = classify(res->val[i].tl, ext_min);
        cls_r[i] = classify(res->val[i].tr, ext_min);
    }
}

int64_t orc_positions(void *handle) { return ((const orc_result *)handle)->positions; }

void orc_free(void *handle) { delete (orc_result *)handle; }


/* ---- cardinality pass (section "Parallel k-mer analysis": the
 * HyperLogLog estimate that sizes the Bloom filter, and the heavy hitters
 * found in the same pass) ----
 *
 * Over every valid window whose key is owned (owner filter as in orc_run):
 *   Hc = fmix64(fmix64(hi ^ kCardSeed) ^ lo);
 *   HyperLogLog (Flajolet, Fusy, Gandouet and Meunier, 2007) with m = 2^p
 *   registers and 64-bit hashes: the top p bits of Hc select register j, and
 *   M[j] is the maximum over the keys of rho = 1 + the number of leading
 *   zeros of the remaining 64 - p bits (64 - p + 1 when they are all zero);
 *   distinct sample: keys whose low `sample_log2` bits of Hc are all zero
 *   are counted exactly;
 *   heavy-hitter sample: the window starting at base index j of the read
 *   set is sampled when the low `heavy_log2` bits of fmix64(j ^ kPosSeed) are
 *   all zero, and sampled windows are counted per key.
 * Results: the registers; the estimate alpha_m m^2 / sum_j 2^-M[j], replaced
 * by m ln(m / V) when it is at most 5m/2 and V > 0 registers are zero (no
 * large-range correction: the hash has 64 bits); the number of sampled keys
 * and of sampled keys with count >= min_depth; the keys whose sampled-window
 * count reaches heavy_min, sorted.
 * Threads take disjoint read ranges; registers merge by maximum (the
 * paper's merge of sketches) and counts by sum. */

typedef struct {
    int32_t k;
    uint32_t flags; /* ORC_FORWARD_ONLY */
    uint32_t n_owners;
    uint32_t owner;
    int32_t hll_p;        /* 4..18 */
    uint32_t sample_log2; /* 0..63 */
    uint32_t heavy_log2;  /* 0..63 */
    uint32_t min_depth;
    uint32_t heavy_min;
    int32_t n_threads;
} orc_card_params_t;

typedef struct {
    double estimate;
    uint64_t sampled_distinct;
    uint64_t sampled_kept;
    uint64_t n_heavy;
    int64_t positions; /* valid windows of owned keys */
} orc_card_result_t;

typedef std::unordered_map<u128, uint64_t, KeyHash> CountMap;

static void card_scan(const uint8_t *ascii, const int64_t *read_off, int64_t r0, int64_t r1,
                      const orc_card_params_t *p, std::vector<uint32_t> &regs, CountMap &sample, CountMap &heavy,
                      int64_t *positions) {
    const int k = p->k, P = p->hll_p;
    const u128 mask = (((u128)1 << (2 * k)) - 1);
    const uint64_t smask = p->sample_log2 ? (~0ULL >> (64 - p->sample_log2)) : 0;
    const uint64_t hmask = p->heavy_log2 ? (~0ULL >> (64 - p->heavy_log2)) : 0;
    int64_t npos = 0;
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t b = read_off[r];
        const int64_t L = read_off[r + 1] - b;
        u128 fwd = 0, rc = 0;
        int64_t run = 0;
        for (int64_t j = 0; j < L; ++j) {
            const int c = code_of(ascii[b + j]);
            if (c == 4) {
                run = 0;
                fwd = rc = 0;
                continue;
            }
            fwd = ((fwd << 2) | (u128)c) & mask;
            rc = (rc >> 2) | ((u128)(3 - c) << (2 * (k - 1)));
            if (++run < k) continue;
            const u128 key = ((p->flags & ORC_FORWARD_ONLY) || fwd <= rc) ? fwd : rc;
            const uint64_t hi = (uint64_t)(key >> 64), lo = (uint64_t)key;
            if (p->n_owners > 1 && orc_owner(hi, lo, p->n_owners) != p->owner) continue;
            ++npos;
            const uint64_t h = key_hash(hi, lo, kCardSeed);
            const uint32_t reg = (uint32_t)(h >> (64 - P));
            const uint64_t rest = h << P;
            const uint32_t rho = rest == 0 ? (uint32_t)(64 - P + 1) : (uint32_t)__builtin_clzll(rest) + 1;
            if (rho > regs[reg]) regs[reg] = rho;
            if ((h & smask) == 0) ++sample[key];
            const int64_t start = b + j - k + 1; /* base index of the window in the read set */
            if ((fmix64((uint64_t)start ^ kPosSeed) & hmask) == 0) ++heavy[key];
        }
    }
    *positions = npos;
}

int orc_card(const uint8_t *ascii, const int64_t *read_off, int64_t n_reads, const orc_card_params_t *p,
             uint32_t *regs_out, orc_card_result_t *res, uint64_t *heavy_hi, uint64_t *heavy_lo, uint64_t heavy_cap) {
    if (!p || p->k < 1 || p->k > 63 || p->hll_p < 4 || p->hll_p > 18 || n_reads < 0) return ORC_EINVAL;
    if (!(p->flags & ORC_FORWARD_ONLY) && (p->k % 2) == 0) return ORC_EINVAL;
    if (p->n_owners < 1 || p->owner >= p->n_owners || p->sample_log2 > 63 || p->heavy_log2 > 63) return ORC_EINVAL;
    const uint32_t T = p->n_threads > 1 ? (uint32_t)p->n_threads : 1u;
    const size_t m = (size_t)1 << p->hll_p;
    std::vector<std::vector<uint32_t>> regs(T, std::vector<uint32_t>(m, 0));
    std::vector<CountMap> sample(T), heavy(T);
    std::vector<int64_t> npos(T, 0);
    auto work = [&](uint32_t t) {
        card_scan(ascii, read_off, n_reads * t / T, n_reads * (t + 1) / T, p, regs[t], sample[t], heavy[t], &npos[t]);
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (uint32_t t = 0; t < T; ++t) th.emplace_back(work, t);
        for (auto &x : th) x.join();
    }
    for (uint32_t t = 1; t < T; ++t) {
        for (size_t j = 0; j < m; ++j) regs[0][j] = std::max(regs[0][j], regs[t][j]);
        for (auto &kv : sample[t]) sample[0][kv.first] += kv.second;
        for (auto &kv : heavy[t]) heavy[0][kv.first] += kv.second;
        npos[0] += npos[t];
    }
    double sum = 0.0;
    uint64_t zeros = 0;
    for (size_t j = 0; j < m; ++j) {
        regs_out[j] = regs[0][j];
        sum += std::ldexp(1.0, -(int)regs[0][j]);
        zeros += regs[0][j] == 0;
    }
    const double md = (double)m;
    const double alpha = m == 16 ? 0.673 : m == 32 ? 0.697 : m == 64 ? 0.709 : 0.7213 / (1.0 + 1.079 / md);
    double e = alpha * md * md / sum;
    if (e <= 2.5 * md && zeros > 0) e = md * std::log(md / (double)zeros);
    res->estimate = e;
    res->sampled_distinct = sample[0].size();
    res->sampled_kept = 0;
    for (auto &kv : sample[0]) res->sampled_kept += kv.second >= p->min_depth;
    std::vector<u128> hv;
    for (auto &kv : heavy[0])
        if (kv.second >= p->heavy_min) hv.push_back(kv.first);
    std::sort(hv.begin(), hv.end());
    res->n_heavy = hv.size();
    for (size_t i = 0; i < hv.size() && i < heavy_cap; ++i) {
        heavy_hi[i] = (uint64_t)(hv[i] >> 64);
        heavy_lo[i] = (uint64_t)hv[i];
    }
    res->positions = npos[0];
    return ORC_OK;
}


/* ---- contig generation (section "Parallel contig generation") ----
 *
 * Input: the UU k-mers (keys with their unique left and right extension
 * bases, as exported).  What is computed:
 *   - a k-mer is read in its key orientation (fwd) or reverse-complemented
 *     (rc); read rc, its right extension is the complement of its stored left
 *     one and vice versa;
 *   - stepping right from an oriented k-mer s with right extension b gives
 *     s' = (s without its first base) + b; s' is looked up by its key; the
 *     step exists when the k-mer is there and its left extension, read in the
 *     orientation of s', is the first base of s (the link agrees from both
 *     ends); stepping left mirrors this;
 *   - every side of a k-mer then has at most one link, so the k-mers form
 *     simple paths and cycles; a step that would leave a k-mer's side and
 *     arrive back at the same side of the same k-mer (a hairpin) is not a link;
 *   - a path is spelled from one end: the first oriented k-mer, then the right
 *     extension of each k-mer before the next; the contig is the smaller of
 *     that string and its reverse complement;
 *   - a cycle of n k-mers is spelled from its smallest key, in fwd
 *     orientation, stepping right: that k-mer and the next n - 1 bases.
 * Contigs are returned sorted.  (Readings listed in the design notes.) */

struct ContigResult {
    std::vector<std::string> seq;
};

namespace {

struct DbgNode {
    u128 key;
    int cl, cr;
};

struct Dbg {
    int k;
    bool fwd_only;
    u128 mask;
    std::vector<DbgNode> nodes;
    std::unordered_map<u128, int64_t, KeyHash> index;

    u128 rc(u128 x) const {
        u128 r = 0;
        for (int i = 0; i < k; ++i) {
            r = (r << 2) | (u128)(3 - (int)(x & 3));
            x >>= 2;
        }
        return r;
    }
    u128 seq(int64_t i, int o) const { return o ? rc(nodes[i].key) : nodes[i].key; }
    int right_ext(int64_t i, int o) const { return o ? 3 - nodes[i].cl : nodes[i].cr; }
    int left_ext(int64_t i, int o) const { return o ? 3 - nodes[i].cr : nodes[i].cl; }
    /* oriented k-mer -> (node, orientation) of its key, or node -1 */
    std::pair<int64_t, int> locate(u128 s) const {
        u128 key = s;
        int o = 0;
        if (!fwd_only) {
            const u128 r = rc(s);
            if (r < s) {
                key = r;
                o = 1;
            }
        }
        auto it = index.find(key);
        return it == index.end() ? std::make_pair((int64_t)-1, 0) : std::make_pair(it->second, o);
    }
    /* step right (dir 0) or left (dir 1) from (i, o) */
    bool step(int64_t i, int o, int dir, int64_t &j, int &o2) const {
        const u128 s = seq(i, o);
        u128 t;
        int back_base;
        if (dir == 0) {
            t = ((s << 2) | (u128)right_ext(i, o)) & mask;
            back_base = (int)(s >> (2 * (k - 1))) & 3;
        } else {
            t = (s >> 2) | ((u128)left_ext(i, o) << (2 * (k - 1)));
            back_base = (int)(s & 3);
        }
        auto f = locate(t);
        if (f.first < 0) return false;
        j = f.first;
        o2 = f.second;
        const int back = dir == 0 ? left_ext(j, o2) : right_ext(j, o2);
        if (back != back_base) return false;
        /* the side left: right side of the key when (dir 0, o 0) or (dir 1, o 1);
           the side reached: left side of the key when (dir 0, o2 0) or (dir 1, o2 1) */
        if (j == i) {
            const int left_side = (dir == 0) == (o == 0) ? 1 : 0;     /* 1: we left through the key's right side */
            const int arrive_right = (dir == 0) == (o2 == 0) ? 0 : 1; /* 1: we arrive at the key's right side */
            if (left_side == arrive_right) return false;             /* hairpin: same side */
        }
        return true;
    }
    std::string spell(u128 s) const {
        std::string out(k, 'A');
        for (int i = k - 1; i >= 0; --i) {
            out[i] = "ACGT"[(int)(s & 3)];
            s >>= 2;
        }
        return out;
    }
};

std::string revcomp_str(const std::string &x) {
    std::string r(x.rbegin(), x.rend());
    for (char &c : r) c = c == 'A' ? 'T' : c == 'C' ? 'G' : c == 'G' ? 'C' : 'A';
    return r;
}

}  // namespace

void *orc_contigs(const uint64_t *key_hi, const uint64_t *key_lo, const uint8_t *cls_l, const uint8_t *cls_r,
                  int64_t n, int32_t k, int32_t forward_only, int64_t *n_contigs) {
    *n_contigs = -1;
    if (k < 1 || k > 63 || n < 0) return nullptr;
    Dbg g;
    g.k = k;
    g.fwd_only = forward_only != 0;
    g.mask = (k == 64) ? ~(u128)0 : (((u128)1 << (2 * k)) - 1);
    g.nodes.resize(n);
    g.index.reserve((size_t)n * 2);
    for (int64_t i = 0; i < n; ++i) {
        if (cls_l[i] > 3 || cls_r[i] > 3) return nullptr; /* not a UU k-mer */
        g.nodes[i] = DbgNode{((u128)key_hi[i] << 64) | key_lo[i], cls_l[i], cls_r[i]};
        g.index[g.nodes[i].key] = i;
    }
    ContigResult *res = new ContigResult();
    std::vector<char> visited(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (visited[i]) continue;
        /* walk left from (i, fwd) to the end of the path, or back to i on a cycle */
        int64_t cur = i, j;
        int o = 0, o2;
        bool cycle = false;
        while (g.step(cur, o, 1, j, o2)) {
            if (j == i) {
                cycle = true;
                break;
            }
            cur = j;
            o = o2;
        }
        if (cycle) {
            /* the cycle's nodes, its smallest key, then spell from there in fwd orientation */
            int64_t m = i, c = i;
            int oc = 0;
            while (g.step(c, oc, 0, j, o2) && j != i) {
                c = j;
                oc = o2;
                if (g.nodes[c].key < g.nodes[m].key) m = c;
            }
            std::string sq = g.spell(g.seq(m, 0));
            visited[m] = 1;
            c = m;
            oc = 0;
            while (g.step(c, oc, 0, j, o2) && j != m) {
                sq.push_back("ACGT"[g.right_ext(c, oc)]);
                c = j;
                oc = o2;
                visited[c] = 1;
            }
            res->seq.push_back(sq);
            continue;
        }
        std::string sq = g.spell(g.seq(cur, o));
        visited[cur] = 1;
        while (g.step(cur, o, 0, j, o2)) {
            sq.push_back("ACGT"[g.right_ext(cur, o)]);
            cur = j;
            o = o2;
            visited[cur] = 1;
        }
        const std::string r = revcomp_str(sq);
        res->seq.push_back(g.fwd_only || sq <= r ? sq : r);
    }
    std::sort(res->seq.begin(), res->seq.end());
    *n_contigs = (int64_t)res->seq.size();
    return res;
}

int64_t orc_contigs_bases(void *handle) {
    int64_t t = 0;
    for (auto &x : ((ContigResult *)handle)->seq) t += (int64_t)x.size();
    return t;
}

/* concatenated contigs (ASCII) and n + 1 offsets */
void orc_contigs_fetch(void *handle, char *seq, int64_t *off) {
    const ContigResult *r = (const ContigResult *)handle;
    int64_t p = 0;
    off[0] = 0;
    for (size_t i = 0; i < r->seq.size(); ++i) {
        memcpy(seq + p, r->seq[i].data(), r->seq[i].size());
        p += (int64_t)r->seq[i].size();
        off[i + 1] = p;
    }
}

void orc_contigs_free(void *handle) { delete (ContigResult *)handle; }

}  /* extern "C" */
