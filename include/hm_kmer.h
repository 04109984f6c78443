/*
 * hm_kmer.h -- C ABI of the MI355X (gfx950) k-mer analysis library.
 *
 * k-mer analysis is the first stage of the Meraculous / HipMer de novo
 * assembly pipeline (arXiv 1705.11147, section "The Meraculous Assembly
 * Pipeline", step 1, and section "Parallel k-mer analysis"): reads are
 * chopped into overlapping k-mers, each distinct k-mer is counted, k-mers
 * seen fewer than a depth threshold are dropped as sequencing errors, two
 * arrays of four counters per k-mer tally the bases seen on its left and
 * right (its "extensions"), and k-mers with a unique high-quality extension
 * on both sides (UU k-mers, section "Parallel contig generation") seed the
 * de Bruijn graph.  A Bloom filter keeps most single-occurrence (erroneous)
 * k-mers out of the count table (section "Parallel k-mer analysis").
 *
 * Conventions shared by every entry point:
 *   - All pointers named in the structs are DEVICE pointers owned by the
 *     caller; the library never allocates or frees device memory, and keeps
 *     no state besides a thread-local error message.
 *   - Calls are asynchronous on `stream` (a hipStream_t, may be NULL for the
 *     legacy default stream).  Argument checks run on the host before any
 *     launch and return HM_EINVAL without touching the device.
 *   - Errors found on the device (table or list full, counter overflow,
 *     export buffer too small) are OR-ed into the caller's status word; read
 *     it with hm_status() after the stream has finished.  A table whose
 *     status is not HM_OK must not be used: rebuild it larger.  Once the
 *     table or list is full, the counting passes skip their remaining work.
 *   - Encoding: A=0, C=1, G=2, T=3; a k-mer of k bases is the 2k-bit
 *     integer with its first base most significant, so numeric order is
 *     lexicographic order.  The key of a k-mer is the smaller of its own and
 *     its reverse complement's encoding (k odd, so they never tie); when the
 *     reverse complement wins, left and right extensions swap sides and are
 *     complemented.  Keys are exported as key_hi = bits 64..125 and
 *     key_lo = bits 0..63.
 *   - Extension classes (one byte per side): 0..3 = the unique base
 *     (A, C, G, T) whose tally reaches ext_min; HM_CLS_FORK = two or more
 *     bases do; HM_CLS_X = none does.
 */
#ifndef HM_KMER_H
#define HM_KMER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HM_ABI_VERSION 2

/* return codes */
#define HM_OK 0
#define HM_EINVAL (-1)     /* bad argument (checked on the host) */
#define HM_ECAPACITY (-2)  /* count table full (probe bound hit) or first-occurrence list full */
#define HM_EHIP (-3)       /* HIP runtime error (launch or copy) */
#define HM_EOUTPUT (-4)    /* export buffer too small; *n_out holds the number needed */
#define HM_EOVERFLOW (-5)  /* a per-k-mer counter would pass 2^32 - 1 */
#define HM_ETIMEOUT (-6)   /* batched form: a phase wait passed its time bound */

/* device status word bits (OR-ed by kernels; hm_status maps them to codes) */
#define HM_ST_TABLE_FULL 1u
#define HM_ST_LIST_FULL 2u
#define HM_ST_OVERFLOW 4u
#define HM_ST_OUTPUT_FULL 8u
#define HM_ST_TIMEOUT 16u
#define HM_ST_DUPLICATE 32u /* hm_contigs: a key appears twice in the input */
#define HM_ST_CLASSIFIED 64u /* not an error: hm_classify_ext has written the table's classification words */
#define HM_ST_STREAM_FULL 128u /* hm_bloom_insert_occ: the occurrence stream had overflowed (see hm_occ_t) */

/* hm_params_t.flags */
#define HM_FORWARD_ONLY 1u /* key = forward encoding (no canonical form); allows even k */
#define HM_BLOOM_BYPASS 2u /* count every occurrence directly, no Bloom test */
#define HM_CHECKED 4u      /* detect counter overflow (needed only past 2^32 positions per table) */
#define HM_BLOOM_IN_TABLE 8u /* the Bloom filter lives in the table (see hm_bloom_t) */

/* hm_export_table flags */
#define HM_EXPORT_UU_ONLY 1u  /* only kept k-mers unique on both sides */
#define HM_EXPORT_ALL 2u      /* every k-mer in the table, also below min_depth */
#define HM_EXPORT_CLASSIFY 4u /* classify while exporting (hm_classify_ext not needed first);
                                 needs the min_depth/ext_min of hm_export_t */
#define HM_EXPORT_SORTED 8u   /* records in ascending key order (key_hi, then key_lo), i.e. the
                                 lexicographic order of the k-mers; needs hm_export_t.sort_work */

#define HM_CLS_FORK 4
#define HM_CLS_X 5

#define HM_SLOT_BYTES 64

/* Packed reads: the output of hm_pack_reads, input of the counting passes.
 * Base i of the concatenated reads is stored
 *   bases2: 2-bit code in word i/32, bits (63 - 2*(i%32)) .. (62 - 2*(i%32));
 *   nmask:  bit (63 - i%64) of word i/64, 1 = not A/C/G/T (window invalid);
 *   hqmask: same position, 1 = valid base with Phred >= qcut.
 * bases2 holds hm_bases2_words(n_bases) words and each mask
 * hm_mask_words(n_bases) words (tail padding included, written by
 * hm_pack_reads). */
typedef struct {
    const uint64_t *bases2;
    const uint64_t *nmask;
    const uint64_t *hqmask;
    const int64_t *read_off; /* n_reads + 1 base offsets, or NULL: read r is [r*read_len, (r+1)*read_len) */
    int64_t n_reads;
    int64_t n_bases;
    int32_t read_len; /* used when read_off is NULL */
} hm_reads_t;

typedef struct {
    int32_t k;          /* 1..63; odd unless HM_FORWARD_ONLY */
    uint32_t min_depth; /* keep k-mers seen >= min_depth times (>= 1; 1 forces HM_BLOOM_BYPASS) */
    uint32_t ext_min;   /* a side's base is a high-quality extension when tallied >= ext_min times (>= 1) */
    /* Owner-computes partition (section "Parallel k-mer analysis"): keep the
     * keys with own(key) == owner (n_owners = 1 keeps all), where
     * own(key) = floor(H * n_owners / 2^64) and
     * H = (key_lo ^ key_hi * 0x9E3779B97F4A7C15) * 0xD1B54A32D192ED03 mod 2^64
     * (multiply-shift hashing).  For n_owners a power of two the
     * owners nest: owner 0 of 2^b is the part of owner 0 of 2^a (a < b) whose
     * H has its top b bits zero. */
    uint32_t n_owners;
    uint32_t owner;
    uint32_t flags;
    uint64_t seed; /* seed of the table and Bloom hashes; the output does not depend on it */
} hm_params_t;

/* Event counters of the counting passes (hm_table_t.stats, HM_N_STATS
 * 64-bit words, added to by every pass; clear them with hm_table_init). */
#define HM_STAT_OCC 0        /* pass 1: valid, owned occurrences */
#define HM_STAT_HIT 1        /* pass 1: k-mer found at the first table lookup */
#define HM_STAT_BLOOM 2      /* pass 1: Bloom test-and-set operations */
#define HM_STAT_DEFER 3      /* pass 1: occurrences sent to the first-occurrence list */
#define HM_STAT_PROBES 4     /* pass 1: table slots inspected */
#define HM_STAT_P2_ENTRIES 5 /* pass 2: list entries processed */
#define HM_STAT_P2_FOUND 6   /* pass 2: entries whose k-mer was in the table */
#define HM_STAT_CAS 7        /* pass 1: compare-and-swap attempts on packed counters */
#define HM_STAT_WIDE 8       /* pass 1: occurrences counted in the wide counters */
#define HM_STAT_HEAVY 9      /* pass 1: occurrences of heavy keys counted in workgroup-local memory */
#define HM_STAT_LINES 10     /* pass 1: table lines inspected (128 bytes: the two slots a probe checks first) */
#define HM_N_STATS 11

#define HM_MAX_HEAVY 256     /* longest heavy-key list of a table */

/* Open-addressing count table of `capacity` 64-byte slots (power of two). */
typedef struct {
    void *slots;
    uint64_t capacity;
    uint32_t max_probe; /* linear-probe bound before HM_ST_TABLE_FULL; 0 = min(4096, capacity) */
    int32_t k;          /* the k the table is built for (set by the caller) */
    uint32_t *status;   /* device status word */
    uint64_t *stats;    /* optional (may be NULL): HM_N_STATS event counters */
    /* Optional heavy hitters (section "Parallel k-mer analysis": very frequent
     * k-mers are accumulated locally, then reduced globally): n_heavy keys as
     * (key_hi, key_lo) pairs in device memory, e.g. from hm_card_summary.  Pass 1
     * counts their occurrences in workgroup-local memory and adds each
     * workgroup's totals to the table once, instead of one atomic per
     * occurrence on the same slot.  Any keys may be listed (a key that never
     * occurs is never inserted); the counts are the same either way. */
    const uint64_t *heavy;
    uint32_t n_heavy;   /* 0..HM_MAX_HEAVY */
    uint32_t reserved;
} hm_table_t;

/* Single-word blocked Bloom filter: n_words 64-bit words (power of two),
 * n_hash bits per key set in one word (1..8).
 * With HM_BLOOM_IN_TABLE there is no separate filter (`words` and `n_words`
 * are ignored): the filter word of a key is the 32-bit classification word of
 * its home slot (the slot its probe sequence starts from), which pass 1 tests
 * and sets with one atomic OR on the table line the probe has just read, so a
 * Bloom test costs no random access of its own.  The filter then has 32 bits
 * per table slot; hm_table_init clears it with the table.  The word is free
 * while counting: hm_classify_ext overwrites it with the slot's classes (only
 * hm_export_table without HM_EXPORT_CLASSIFY reads them) and sets
 * HM_ST_CLASSIFIED; a later pass 1 into the same table, whose filter bits are
 * then gone, inserts every absent k-mer instead of testing the filter (the
 * counts stay exact, the table takes the singletons too).  Counts never
 * depend on the filter. */
typedef struct {
    uint64_t *words;
    uint64_t n_words;
    uint32_t n_hash;
} hm_bloom_t;

/* First-occurrence list between the two counting passes: one entry per
 * occurrence that the Bloom filter had not seen (key: 2 words, ext: 1 byte).
 * Optional presence filter: pass 1 sets present_hash bits of every k-mer it
 * inserts into the table in one word of `present` (n_words a power of two),
 * and pass 2 skips the table lookup of entries whose bits are not all set
 * (those k-mers were never inserted).  Sized near the number of table keys
 * it stays cache-resident; it never changes the output. */
typedef struct {
    uint64_t *keys;  /* 2 * capacity words */
    uint8_t *ext;    /* capacity bytes */
    uint64_t capacity;
    uint64_t *count; /* device counter of entries (zeroed by hm_list_init) */
    uint64_t *present;      /* optional (may be NULL) */
    uint64_t present_words; /* power of two when present != NULL */
    uint32_t present_hash;  /* bits per k-mer, 1..8 */
} hm_list_t;

/* Export destination: structure-of-arrays records. */
typedef struct {
    uint64_t *key_hi;
    uint64_t *key_lo;
    uint32_t *count;
    uint32_t *tl; /* 4 per record */
    uint32_t *tr; /* 4 per record */
    uint8_t *cls_l;
    uint8_t *cls_r;
    uint64_t capacity;
    uint64_t *n_out;  /* device counter: records exported (or needed, on HM_EOUTPUT) */
    uint64_t *digest; /* optional (may be NULL): 2 words, order-free sum and xor of per-record hashes */
    uint32_t min_depth; /* used with HM_EXPORT_CLASSIFY */
    uint32_t ext_min;   /* used with HM_EXPORT_CLASSIFY */
    void *sort_work;          /* used with HM_EXPORT_SORTED: device scratch, 256-byte aligned, */
    uint64_t sort_work_bytes; /* at least hm_export_sort_bytes(capacity) bytes; else may be NULL / 0 */
} hm_export_t;

/* ---- sizes and helpers ------------------------------------------------ */

int hm_abi_version(void);
const char *hm_last_error(void);
uint64_t hm_bases2_words(int64_t n_bases);
uint64_t hm_mask_words(int64_t n_bases);
size_t hm_table_bytes(uint64_t capacity);
size_t hm_bloom_bytes(uint64_t n_words);
size_t hm_list_bytes(uint64_t capacity);
/* Scratch that hm_export_table needs with HM_EXPORT_SORTED for an export
 * buffer of `capacity` records: 88 bytes per record (keys, record index and
 * the staged counters, double-buffered where a counting pass needs it), plus
 * 1 KiB per 4096 records and about 257 KiB of digit and group tables. */
size_t hm_export_sort_bytes(uint64_t capacity);
/* Host-only argument check of a parameter block (no device access). */
int hm_check_params(const hm_params_t *p);

/* Fill a table with empty slots and clear its status word (and stats). */
int hm_table_init(hm_table_t *t, hipStream_t stream);
/* Clear a Bloom filter. */
int hm_bloom_init(hm_bloom_t *b, hipStream_t stream);
/* Clear a first-occurrence list's counter (and its presence filter). */
int hm_list_init(hm_list_t *l, hipStream_t stream);
/* Synchronize `stream`, read the status word and map it to a return code. */
int hm_status(const hm_table_t *t, hipStream_t stream);
/* Map a status word the caller has already copied to the host (for instance
 * with an asynchronous copy into pinned memory, so that a host thread serving
 * many streams never blocks on one) to the code hm_status would return, with
 * the same error message.  Touches no device; never fails itself. */
int hm_status_code(uint32_t status);

/* ---- the k-mer analysis path ------------------------------------------ */

/* Pack reads: ascii[n_bases] bases (A/C/G/T in either case; anything else
 * invalid) and qual[n_bases] Phred bytes (numeric Phred = byte - qual_offset)
 * into the 2-bit and mask words described at hm_reads_t.  Read boundaries
 * are not needed here (the layout is per base).  Section "Parallel k-mer
 * analysis" (reading the reads); the quality gate implements the
 * high-quality-extension reading (a base is tallied only at Phred >= qcut). */
int hm_pack_reads(const uint8_t *ascii, const uint8_t *qual, int64_t n_bases, uint8_t qual_offset, uint8_t qcut,
                  uint64_t *bases2, uint64_t *nmask, uint64_t *hqmask, hipStream_t stream);

/* Counting pass 1 (section "Parallel k-mer analysis", Bloom filter
 * paragraph): every valid k-mer occurrence (canonical, owner-filtered) is
 * looked up in the table; if present it is counted with its extensions.  An
 * absent k-mer tests and sets its bits in the Bloom filter with one atomic OR
 * on one word: if the filter had already seen it, the k-mer is inserted and
 * this occurrence counted; otherwise the occurrence is appended to the
 * first-occurrence list `l`.
 * With HM_BLOOM_IN_TABLE the word is the home slot's (see hm_bloom_t) and
 * `b` only supplies n_hash.
 * With HM_BLOOM_BYPASS (or min_depth == 1) every occurrence is counted and
 * `b`/`l` may be NULL.  `t` must be initialized; `l` must be initialized
 * before the first pass-1 call of a table (several read batches may be
 * passed through pass 1 one after another). */
int hm_bloom_insert(const hm_reads_t *r, const hm_params_t *p, hm_bloom_t *b, hm_table_t *t, hm_list_t *l,
                    hipStream_t stream);

/* Counting pass 2 (section "Parallel k-mer analysis": the Bloom filter
 * paragraph, where a k-mer the filter has seen is inserted so that the count
 * table then counts it; read here so that every occurrence is counted
 * exactly once): each first-occurrence entry of `l` whose k-mer is in the
 * table (i.e. was seen at least twice, or is a Bloom false positive) is
 * counted with its extensions.  After it the table holds, for every k-mer
 * with count >= 2, exactly its count and extension tallies over all
 * occurrences, whatever the Bloom false positives were.  `r` is unused by
 * the current design and may be NULL. */
int hm_kmer_count(const hm_reads_t *r, const hm_params_t *p, hm_table_t *t, hm_list_t *l, hipStream_t stream);

/* Depth filter and extension classification (sections "Parallel k-mer
 * analysis": epsilon cutoff and t_hq; "The Meraculous Assembly Pipeline":
 * forks; "Parallel contig generation": UU only): for every occupied slot,
 * count = total occurrences, kept = count >= min_depth, and each side gets
 * its class byte.  Results stay in the table for hm_export_table. */
int hm_classify_ext(const hm_params_t *p, hm_table_t *t, hipStream_t stream);

/* Export (section "Parallel contig generation": only the UU k-mers, those
 * with a unique high-quality extension on both sides, go on to build the de
 * Bruijn graph; section "The Meraculous Assembly Pipeline", step 1: the
 * k-mers that survive the depth filter, with their extensions).
 * Stream-compact the classified table into `out`.  flags: HM_EXPORT_UU_ONLY,
 * HM_EXPORT_ALL, HM_EXPORT_CLASSIFY, HM_EXPORT_SORTED.  Zeroes out->n_out (and
 * out->digest) first.  Without HM_EXPORT_SORTED the records come in no fixed
 * order: each run of 2048 table slots takes its output range with one atomic,
 * so runs land in the order they finish, each in slot (hash) order; the set of
 * records and the digest do not depend on it.  With HM_EXPORT_SORTED they are
 * in ascending key order: a radix sort of
 * the 2k key bits runs after the compaction on the same
 * stream and uses out->sort_work as scratch (HM_EINVAL if it is NULL,
 * misaligned, smaller than hm_export_sort_bytes(out->capacity), or if
 * out->capacity >= 2^32).  The digest does not depend on the order.  After
 * an HM_EOUTPUT failure the partial records are sorted too, and stay invalid.
 * The sort groups records by their top 16 key bits with two stable counting
 * passes and then orders each group in one workgroup (keys of 32 bits or
 * more), or takes a counting pass per 8 key bits (shorter keys). */
int hm_export_table(const hm_table_t *t, uint32_t flags, hm_export_t *out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * hm_export_table whose key-ordered export (HM_EXPORT_SORTED) takes its
 * scratch from an array the library holds on each GPU instead of
 * out->sort_work (out->sort_work and out->sort_work_bytes are ignored).
 * Limit: out->capacity <= HM_EXPORT_STATIC_MAX_RECORDS (2^18 records; the
 * array is 24 MiB per GPU, held from the library's load on that GPU until the
 * process ends); a larger capacity returns HM_EINVAL before any device work.
 * Nothing is allocated.  The first call on a device looks up the array's
 * address there (make one call before capturing a graph).  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents (each
 * call writes what it reads, so nothing needs clearing): calls that overlap
 * on one GPU (two streams, two host threads) race and give wrong records.
 * Without HM_EXPORT_SORTED it is hm_export_table.  Output equals
 * hm_export_table's with a caller scratch. */
#define HM_EXPORT_STATIC_MAX_RECORDS (1u << 18)
int hm_export_table_static(const hm_table_t *t, uint32_t flags, hm_export_t *out, hipStream_t stream);


/* ---- cardinality pass: sizing and heavy hitters, before pass 1 -------- */

/* Section "Parallel k-mer analysis": a first pass over the reads estimates
 * the number of distinct k-mers with HyperLogLog (64-bit hashes; sketches
 * merge by keeping the larger register) so that the Bloom filter can be sized,
 * and finds the very frequent k-mers (heavy hitters) in the same pass.  Over
 * every valid window whose key is owned (hm_params_t owner filter):
 *   Hc = fmix64(fmix64(key_hi ^ 0xB7E151628AED2A6A) ^ key_lo)  (fmix64: the
 *        64-bit finalizer of MurmurHash3);
 *   HyperLogLog (Flajolet, Fusy, Gandouet, Meunier 2007), m = 2^hll_p
 *        registers: the top hll_p bits of Hc pick register j, which keeps the
 *        maximum of 1 + the leading-zero count of the other 64 - hll_p bits
 *        (64 - hll_p + 1 when they are all zero);
 *   distinct sample: a key whose Hc has `sample_log2` low zero bits is
 *        counted in `sample` (every occurrence), so the sample's keys with
 *        count >= min_depth, times 2^sample_log2, estimate the kept k-mers;
 *   window sample: the window starting at base index j of the read set is
 *        counted in `heavy` when fmix64(j ^ 0x452821E638D01377) has
 *        `heavy_log2` low zero bits; a key with many sampled windows is a
 *        heavy hitter.
 * The result depends only on the reads, not on the order of work. */
typedef struct {
    uint32_t *registers;  /* 2^hll_p registers, device */
    int32_t hll_p;        /* 4..16 */
    uint32_t sample_log2; /* 0..63 */
    uint32_t heavy_log2;  /* 0..63 */
    uint32_t reserved;
    uint64_t *positions;  /* device counter: valid windows of owned keys */
    hm_table_t sample;    /* count table of the distinct sample (k as in the params) */
    hm_table_t heavy;     /* count table of the window sample */
} hm_card_t;

/* Summary of a cardinality pass (written to device memory by hm_card_summary). */
typedef struct {
    double estimate;           /* HyperLogLog estimate of distinct owned k-mers: alpha_m m^2 / sum 2^-M[j],
                                  or m ln(m / V) when that is <= 5m/2 and V > 0 registers are zero */
    uint64_t sampled_distinct; /* keys in the distinct sample */
    uint64_t sampled_kept;     /* of those, keys with count >= min_depth */
    uint64_t n_heavy;          /* keys whose window-sample count >= heavy_min (all, also past heavy_cap) */
    uint64_t positions;        /* valid windows of owned keys */
} hm_card_summary_t;

/* Zero the registers and the position counter, and initialize both tables. */
int hm_card_init(hm_card_t *c, hipStream_t stream);

/* Add one batch of packed reads to the sketch (call once per batch, after
 * hm_card_init).  A table that fills up sets HM_ST_TABLE_FULL in its status
 * word (hm_status then reports HM_ECAPACITY); the registers and the position
 * count stay exact. */
int hm_cardinality(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hipStream_t stream);

/* Reduce the sketch to `out` (device memory): the estimate, the distinct
 * sample's size and its keys with count >= min_depth, and the heavy hitters,
 * i.e. keys whose window-sample count >= heavy_min; the first heavy_cap of
 * them (in no particular order) are written to heavy_keys as (key_hi,
 * key_lo) pairs, 2 * heavy_cap words of device memory (may be NULL when
 * heavy_cap is 0). */
int hm_card_summary(const hm_card_t *c, uint32_t min_depth, uint32_t heavy_min, uint64_t *heavy_keys,
                    uint64_t heavy_cap, hm_card_summary_t *out, hipStream_t stream);


/* ---- owned-occurrence stream: the sharded shape --------------------------
 *
 * Section "Parallel k-mer analysis" (owner computes): a processor keeps only
 * the k-mers it owns, a small share of all windows.  A pass 1 over the reads
 * would scan every window again to find that share after the cardinality
 * pass has already found it, so the cardinality pass can write the owned
 * occurrences out as it meets them, and pass 1 then reads that stream
 * instead of the reads.  The table, and so the output, are the same as with
 * hm_bloom_insert over the same reads and owner filter.
 *
 * Entries come in no fixed order: each wave of the cardinality pass reserves
 * chunks of 1024 entries with one atomic add on `count` and fills them in
 * order, up to 64 entries per write; the unused tail of a wave's last chunk of
 * a launch is marked as holes (ext byte 0xFF), which pass 1 skips.  So *count (entries reserved,
 * holes included) exceeds the owned occurrences by at most 1023 per wave of
 * each hm_cardinality_occ launch (4 waves per workgroup, 4 workgroups per CU).
 * If *count passes `capacity`, the entries past it were dropped: the stream
 * is void (hm_bloom_insert_occ then sets HM_ST_STREAM_FULL and counts
 * nothing), and the caller reruns with a larger stream. */
typedef struct {
    uint64_t *keys;    /* 2 * capacity words, 16-byte aligned: entry i is (key_hi, key_lo) at keys[2i], keys[2i+1] */
    uint8_t *ext;      /* capacity bytes: left | right << 4, 0..3 = base, 4 = no extension; 0xFF = hole */
    uint64_t capacity; /* entries */
    uint64_t *count;   /* device counter of entries reserved (zeroed by hm_occ_init) */
} hm_occ_t;

size_t hm_occ_bytes(uint64_t capacity); /* 17 bytes per entry */

/* Zero the stream's entry counter. */
int hm_occ_init(hm_occ_t *o, hipStream_t stream);

/* hm_cardinality, and in the same scan append every valid window whose key
 * is owned (hm_params_t owner filter) to `o` as (canonical key, extension
 * byte), with the extensions as pass 1 takes them (HQ neighbours, swapped and
 * complemented when the reverse complement is the key).  Call once per read
 * batch after hm_card_init and hm_occ_init; the batches' entries accumulate
 * in one stream.  HM_EINVAL for a NULL or misaligned stream. */
int hm_cardinality_occ(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hm_occ_t *o, hipStream_t stream);

/* Counting pass 1 (as hm_bloom_insert) over the occurrences of a stream
 * written by hm_cardinality_occ instead of over reads: every entry
 * [0, *o->count) that is not a hole is looked up, counted, inserted or
 * deferred to `l` exactly as hm_bloom_insert does with the same occurrence.
 * The owner filter was applied when the stream was written (p->n_owners and
 * p->owner are not used again); k, flags, seed and min_depth are.  Then
 * hm_kmer_count, hm_classify_ext and hm_export_table as usual.  If the stream
 * overflowed (*count > capacity) the pass sets HM_ST_STREAM_FULL in the
 * table's status and does nothing else; hm_status reports HM_ECAPACITY. */
int hm_bloom_insert_occ(const hm_occ_t *o, const hm_params_t *p, hm_bloom_t *b, hm_table_t *t, hm_list_t *l,
                        hipStream_t stream);


/* ---- binned counting: owner computes inside one GPU -------------------
 *
 * Section "Parallel k-mer analysis" gives every k-mer an owner by a hash of
 * the k-mer; each occurrence travels to its owner, which filters its share
 * with a Bloom filter and counts it in a hash table of its own.  The binned
 * path makes the owners bins small enough for one workgroup's local memory:
 *   hm_bin_kmers   partitions the occurrences of a read set by a hash of the
 *                  canonical key into 2^(group_bits + bin_bits) bins of
 *                  16-byte records (two counting-sort passes with exact
 *                  offsets from histograms);
 *   hm_count_bins  runs, per bin and in local memory, the two-pass method of
 *                  hm_bloom_insert / hm_kmer_count (an occurrence of a k-mer in
 *                  the bin's table is counted; an absent k-mer tests and sets
 *                  its bits in the bin's Bloom filter, and is inserted and
 *                  counted if the filter had seen it, else deferred and
 *                  counted after the bin's last occurrence if its k-mer is in
 *                  the table by then), then the depth filter, classification
 *                  and export of hm_export_table with HM_EXPORT_CLASSIFY.
 * A bin whose keys would fill its local table past three quarters (more
 * than 384 k-mers inserted) or whose deferred occurrences pass 2048 is not
 * counted there: its records go whole to an occurrence stream, which the
 * global-table path counts (hm_bloom_insert_occ, hm_kmer_count,
 * hm_export_table into a second buffer), and hm_export_merge appends that
 * export to the binned one.  The records and the digest are those of the
 * global-table path over the same reads; the order differs.
 *
 * Limits: fixed-length reads (read_off NULL) of at most 16320 bases, k <= 61
 * (the key and its two extension codes share a 16-byte record), at most 2^21
 * bins, fewer than 2^32 records (windows and padding) per call. */

/* Event counters of hm_count_bins (hm_bins_t.stats, HM_N_BIN_STATS 64-bit words). */
#define HM_BIN_STAT_RECORDS 0     /* records (valid, owned windows) in the bins */
#define HM_BIN_STAT_SPILLED_BINS 1 /* bins sent to the occurrence stream */
#define HM_BIN_STAT_SPILLED 2     /* records sent to the occurrence stream */
#define HM_BIN_STAT_DEFERRED 3    /* occurrences deferred by the bins' Bloom filters (bins counted locally) */
#define HM_BIN_STAT_KEYS 4        /* k-mers inserted into the bins' local tables */
#define HM_BIN_STAT_KEPT 5        /* records exported from the local tables */
#define HM_N_BIN_STATS 6

typedef struct {
    uint64_t *recs;      /* 2 * capacity words, 128-byte aligned: the records, bin after bin */
    uint64_t *tmp;       /* 2 * capacity words, 128-byte aligned: the first partition level's output, a region
                            per first-level workgroup holding a piece per group (the top group_bits of the bin)
                            (scratch of hm_bin_kmers / hm_bin_occ; free afterwards, e.g. as the keys of the
                            spill stream) */
    uint64_t capacity;   /* records: at least hm_bins_capacity(windows, group_bits, bin_bits) */
    uint32_t group_bits; /* 0..10 */
    uint32_t bin_bits;   /* 0..11: bins = 2^(group_bits + bin_bits) */
    uint64_t *scratch;   /* hm_bins_scratch_bytes(group_bits, bin_bits) bytes, 16-byte aligned */
    uint64_t *bin_start; /* 2^(group_bits + bin_bits) + 1 words: bin i holds records [bin_start[i], bin_start[i+1]) */
    uint32_t *status;    /* device status word (cleared by hm_bin_kmers) */
    uint64_t *stats;     /* optional (may be NULL): HM_N_BIN_STATS counters (cleared by hm_bin_kmers) */
} hm_bins_t;

/* Scratch bytes of hm_bin_kmers and hm_count_bins: for 2^g groups and 2^(g+b) bins,
 * 2^27 + 8 * (2050 + 2 * 2^g) + 4096 * 2^g + 32 * 2^(g+b) bytes (the 128 MiB are where
 * hm_count_bins stages each workgroup's records before it takes their output
 * range with one atomic add); 0 if g is above 10 or b above 11. */
size_t hm_bins_scratch_bytes(uint32_t group_bits, uint32_t bin_bits);

/* Records the bins need room for (hm_bins_t.capacity) for a read set of `windows`
 * windows: the windows plus the padding that makes every destination range a
 * whole number of the blocks the partition writes whole (8 records, 128 bytes,
 * in the first level; 4 records, 64 bytes, in the second),
 * windows + max(7 * 1024 * 2^g, 3 * 8 * 2^(g+b)); 0 if g is above 10 or b
 * above 11.  Padding records ("holes": extension field 63) sit at the ends of
 * ranges and are skipped. */
uint64_t hm_bins_capacity(uint64_t windows, uint32_t group_bits, uint32_t bin_bits);

/* Partition every valid window of `r` whose key is owned (hm_params_t
 * owner filter) into the bins of `b`: record = (key_lo, key_hi | ext << 58),
 * ext = left | right << 3 with the extensions as pass 1 takes them.  The bin
 * of a key is the top group_bits + bin_bits bits of
 * (key_lo ^ key_hi * 0xC2B2AE3D27D4EB4F) * 0x165667B19E3779F9 mod 2^64
 * (multiply-shift hashing).  flags: 0, or HM_BINS_COUNTED when
 * hm_cardinality_bins has counted the first level's histogram for these
 * reads, params and bins, on the same stream, with no hm_bin_kmers on these
 * bins' scratch since (the partition then starts from it; the library notes
 * each hm_cardinality_bins on the host and checks the note).  HM_EINVAL
 * (nothing launched) for unknown flags, HM_BINS_COUNTED without such a
 * note, variable-length reads, k > 61, b->capacity below hm_bins_capacity,
 * or 2^32 or more records. */
#define HM_BINS_COUNTED 1u
int hm_bin_kmers(const hm_reads_t *r, const hm_params_t *p, hm_bins_t *b, uint32_t flags, hipStream_t stream);

/* hm_bin_kmers over an owned-occurrence stream (hm_cardinality_occ's output:
 * one owner's share of a sharded run, section "Parallel k-mer analysis")
 * instead of over the reads: every entry of `o` but its holes becomes a
 * record in its bin, as hm_bin_kmers would place it; hm_count_bins and
 * hm_export_merge follow as after hm_bin_kmers.  The stream must be whole (its
 * count not past its capacity; an overflowed stream's dropped entries are not
 * there).  b->capacity: at least hm_bins_capacity(o->capacity, ...).
 * HM_EINVAL (nothing launched) for k > 61, bins too small for the stream's
 * capacity, or a capacity of 2^32 or more records with the padding. */
int hm_bin_occ(const hm_occ_t *o, const hm_params_t *p, hm_bins_t *b, hipStream_t stream);

/* hm_cardinality (section "Parallel k-mer analysis": the HyperLogLog pass that
 * sizes the filters), also counting, for each workgroup of hm_bin_kmers' first
 * level, how many owned windows of each group its tiles hold: the histogram
 * hm_bin_kmers would otherwise count in a pass of its own.  Call it with the
 * same reads, params and bins (group_bits, bin_bits) right before
 * hm_bin_kmers(..., HM_BINS_COUNTED, ...), which then skips that pass; the
 * histogram lives in the bins' scratch until that hm_bin_kmers consumes it.
 * The sketch it leaves is the same as hm_cardinality's.  HM_EINVAL: reads of
 * variable length, or 2^hll_p + 4 * 2^group_bits above 65536 (the pass keeps
 * the registers and the group counters in one workgroup's memory). */
int hm_cardinality_bins(const hm_reads_t *r, const hm_params_t *p, hm_card_t *c, hm_bins_t *b, hipStream_t stream);

/* Count the bins of `b` (after hm_bin_kmers with the same params) and export
 * every k-mer with count >= p->min_depth, classified with p->ext_min, into
 * `out` (only the UU k-mers with flags = HM_EXPORT_UU_ONLY; no other flag).
 * Zeroes out->n_out, out->digest and spill->count first.  The records of bins
 * that do not fit in local memory go to `spill` (no holes; spill->keys may be
 * b->tmp, whose capacity suffices); count them with the global-table path
 * and hm_export_merge.  Device errors in b->status: HM_ST_OUTPUT_FULL (out
 * too small: *out->n_out holds the number needed), HM_ST_STREAM_FULL (spill
 * too small).  Bloom bypass (HM_BLOOM_BYPASS or min_depth == 1) inserts every
 * k-mer, so bins then take fewer distinct k-mers before spilling. */
int hm_count_bins(const hm_bins_t *b, const hm_params_t *p, uint32_t flags, hm_export_t *out, hm_occ_t *spill,
                  hipStream_t stream);

/* Append src's records [0, *src->n_out) to dst after its *dst->n_out
 * records, add the record counts and combine the digests (sum added, xor
 * xor-ed).  Both run on `stream`; a dst too small sets HM_ST_OUTPUT_FULL in
 * *status (dst's count then holds the number needed). */
int hm_export_merge(const hm_export_t *src, hm_export_t *dst, uint32_t *status, hipStream_t stream);


/* ---- contig generation (section "Parallel contig generation") ---------- */

/* The UU k-mers form the de Bruijn graph: a k-mer's two-letter value names
 * the base before and after it, so a contig grows by looking up the k-mer
 * spelled by its last k-1 bases and its extension, until a lookup fails.
 * Two UU k-mers are linked when the extension of each spells the other
 * (keys are canonical: a k-mer read reverse-complemented has the complement
 * of its stored left extension on its right, and vice versa; a link from a
 * side of a k-mer back to the same side is not one).  Every side then has at
 * most one link, so the k-mers form simple paths and cycles, and the contigs
 * are unique: a path is spelled from one end (its first k-mer, then one base
 * per further k-mer) and given as the smaller of that string and its
 * reverse complement; a cycle of n k-mers is spelled from its smallest key,
 * read in key orientation, stepping right: k + n - 1 bases.  With
 * HM_FORWARD_ONLY keys are forward k-mers and no reverse complement is taken.
 *
 * The paper grows subcontigs from random seeds with remote atomics to settle
 * two walkers meeting; here every k-mer finds its successor at once and the
 * paths are ranked by pointer jumping (log-depth, no seeds), which gives the
 * same contigs. */
typedef struct {
    uint8_t *seq;          /* contig bases (ASCII A, C, G, T), concatenated */
    uint64_t seq_capacity; /* bytes of seq */
    uint64_t *off;         /* contig c is seq[off[c], off[c + 1]); off_capacity + 1 entries */
    uint64_t off_capacity; /* most contigs */
    uint64_t *counts;      /* device, 2 words: contigs and bases (the numbers needed, on overflow) */
    uint32_t *status;      /* device status word: HM_ST_OUTPUT_FULL, HM_ST_DUPLICATE, HM_ST_TABLE_FULL */
    void *work;            /* device scratch, 256-byte aligned, at least hm_contigs_work_bytes(uu capacity) */
    uint64_t work_bytes;
} hm_contigs_t;

/* Scratch of hm_contigs for an input of up to `capacity` records: 186 bytes
 * per record (two 32-byte index slots, so the index is at most half full; and
 * for each of the k-mer's two readings its links, ranks, segment and list
 * entries), plus 512 bytes; 0 if capacity is 2^29 or more. */
size_t hm_contigs_work_bytes(uint64_t capacity);

/* Contigs of the UU k-mers among the records of `uu` (an export: key_hi,
 * key_lo, cls_l, cls_r of min(*uu->n_out, uu->capacity) records, in any
 * order, keys distinct; records whose class on either side is not a base
 * (0..3) are not part of the graph; other fields unused; capacity < 2^29).
 * k and flags (HM_FORWARD_ONLY) as for the counting passes.  Clears
 * out->counts and out->status first.  Contig c occupies seq[off[c],
 * off[c + 1]); contigs come in no particular order, and off[counts[0]] =
 * counts[1].  Asynchronous on `stream`, no host synchronization: the pointer
 * jumping stops on the device.  Returns HM_EINVAL on bad arguments (nothing
 * launched).  After the stream, out->status reports HM_ST_OUTPUT_FULL (more
 * contigs or bases than the capacities: counts hold the numbers needed, the
 * output is invalid) or HM_ST_DUPLICATE (a key appears twice: no output);
 * HM_ST_TIMEOUT would mean a ranking bound was not enough (not expected). */
int hm_contigs(const hm_export_t *uu, int32_t k, uint32_t flags, hm_contigs_t *out, hipStream_t stream);


/* ---- batched form: many read sets, one persistent launch -------------- */

/* One read set of a batch: fixed-length reads (read_len <= 16320), its own
 * packed-read buffers, count table, Bloom filter, first-occurrence list and
 * export destination (all device memory owned by the caller, sized as for
 * the plain path).  The table's k must equal the batch's params.k. */
typedef struct {
    const uint8_t *ascii;
    const uint8_t *qual;
    int64_t n_reads;
    int32_t read_len;
    uint64_t *bases2; /* hm_bases2_words(n_reads * read_len) words */
    uint64_t *nmask;  /* hm_mask_words(n_reads * read_len) words */
    uint64_t *hqmask;
    hm_table_t table;
    hm_bloom_t bloom; /* unused with HM_BLOOM_BYPASS or min_depth == 1 */
    hm_list_t list;   /* likewise */
    hm_export_t out;
} hm_batch_set_t;

/* Launch shape of the persistent kernel (chosen by an autotuner). */
typedef struct {
    int32_t blocks_per_cu;  /* persistent grid = CUs x blocks_per_cu, 1..16 */
    int32_t tile_bases;     /* bases of reads per pass-1 work item, 1024..262144 (staged 16384 at a time) */
    int32_t list_per_item;  /* first-occurrence entries per pass-2 work item, >= 256 */
    int32_t slots_per_item; /* table slots per classify+export work item, multiple of 2048 */
    int32_t set_major;      /* 0: all pass-1 items first, then all pass-2 items; n >= 1: set by set, each
                               set's pass 2 after the pass 1 of the (n-1)-th following set (few tables live
                               at once, and pass-2 items rarely wait for their set's pass-1 tail) */
} hm_batch_tuning_t;

/* Host-side plan returned by hm_batch_prepare and consumed by hm_batch_launch. */
typedef struct {
    void *work;         /* caller's device scratch holding descriptors and counters */
    int32_t n_sets;
    int32_t grid;       /* persistent-kernel blocks */
    int64_t n_items;    /* work items over all phases and sets */
    int64_t n_regions;  /* buffers cleared at launch */
    int64_t pack_words; /* mask words packed at launch, over all sets */
    int32_t k;
    int32_t reserved;
} hm_batch_plan_t;

/* Device scratch a batch of n_sets needs. */
size_t hm_batch_work_bytes(int32_t n_sets);

/* Validate the sets, lay out their descriptors and work items (larger sets
 * first; ordered set by set or phase by phase as tuning.set_major says; a
 * set's pass-2 items always come after its pass-1 items; export ranges
 * separately).  A wave's first-occurrence list chunk persists across work
 * items of one set, so each set's list needs CUs x blocks_per_cu x 4 x 255
 * entries of slack beyond its distinct k-mers.
 * and copy them into `work` (device, >= hm_batch_work_bytes(n_sets)).
 * Synchronizes `stream`; not capturable.  Sections as for the plain path. */
int hm_batch_prepare(const hm_batch_set_t *sets, int32_t n_sets, const hm_params_t *p, uint8_t qual_offset,
                     uint8_t qcut, uint32_t export_flags, const hm_batch_tuning_t *tuning, void *work,
                     size_t work_bytes, hm_batch_plan_t *plan, hipStream_t stream);

/* Run the whole path for every set of a prepared batch: clear tables,
 * filters, lists and counters; pack all reads; one persistent kernel whose
 * blocks take counting work items from an atomic ticket (a pass-2 item of a
 * set waits for all pass-1 items of that set: agent-scope release/acquire on
 * per-set counters); then classify and export every set.
 * Results land in each set's export buffers, and per-set status words as
 * in the plain path (plus HM_ST_TIMEOUT if a wait passed its bound).
 * Launches kernels only (no copies, no allocation): capturable in a HIP
 * graph and replayable.  Output equals the plain path's, set by set. */
int hm_batch_launch(const hm_batch_plan_t *plan, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HM_KMER_H */
