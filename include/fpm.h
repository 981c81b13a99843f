/*
 * fpm.h -- C ABI of the fingerprint-filtered approximate dictionary matcher
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Cislak & Grabowski, "Lightweight Fingerprints for Fast Approximate
 * Keyword Matching Using Bitwise Operations" (arXiv:1711.08475).
 *
 *   Problem (Section 1): a query P is compared against every word of a
 *   collection D = [S_1 .. S_|D|]; report every word within Hamming or
 *   Levenshtein distance k.
 *   Fingerprints (Section 3, construction in Section 3.2): a fixed-size bit
 *   block per string -- occurrence, occurrence halved, count (b = 2 bits per
 *   symbol, saturating) or position (p = 3 bits per symbol, first position,
 *   all ones when >= 2^p - 1 or absent, leftover bits are occurrence bits).
 *   Comparison (Section 3.3, Eq. 1): D(S1, S2) >= ceil(F_D / 2), so a pair is
 *   rejected without verification when F_D > 2k (bigram fingerprints: 4k).  Survivors are verified
 *   exactly (Ham: mismatches up to k + 1; Lev: the 2k+1 band).
 *
 * Readings fixed by this library where the paper is silent or inconsistent:
 *   - field j of the symbol map occupies the j-th lowest bits of the
 *     fingerprint (occ: bit j; count: bits 2j..2j+1 holding the binary count;
 *     pos: bits 3j..3j+2, occurrence bits after the position fields; occh:
 *     bit 2j first half, bit 2j+1 second half);
 *   - count F_D is the L1 distance of the saturated counts (the literal
 *     Hamming weight of the XOR can reject true matches: "eet" vs "ett");
 *   - pos F_D is the number of differing position fields plus the Hamming
 *     weight of the XOR of the occurrence bits;
 *   - 16-bit fingerprints hold 16 occ / 8 count / 8 occh / 5 pos + 1 occ
 *     symbols (Section 4), 32-bit ones 32 / 16 / 16 / 10 + 2;
 *   - common / rare / mixed symbol sets rank symbols by total occurrences in
 *     the dictionary, ties by byte value; mixed takes ceil(F/2) most frequent
 *     then floor(F/2) least frequent; the i-th chosen symbol gets field i.
 *
 * Strings are byte strings of length 0..255 given in CSR form: `bytes`
 * holds them back to back, string i is bytes[offsets[i] .. offsets[i+1]),
 * offsets has n + 1 non-decreasing entries.  Query and word indices in
 * results are positions in the caller's lists.
 *
 * Errors: every entry point returns an fpm_status; on failure a message is
 * kept per thread and fpm_last_error() returns it.  FPM_EINVAL: a null
 * pointer, decreasing offsets, a string longer than 255, bits not 16 or 32, a
 * custom map entry >= the variant's field count, a bad option.
 * FPM_EUNSUPPORTED: position or occurrence-halved fingerprints with the
 * Levenshtein metric (Section 3 restricts both to Hamming), k outside 1..3
 * for matching.  FPM_ENOMEM / FPM_EDEVICE: a HIP allocation or launch failed.
 *
 * Threads: an index is immutable after it is built and may be shared by
 * threads; a plan is owned by one thread at a time.
 */
#ifndef FPM_H
#define FPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPM_OK = 0,
    FPM_EINVAL = -1,
    FPM_EUNSUPPORTED = -2,
    FPM_ENOMEM = -3,
    FPM_EDEVICE = -4
} fpm_status;

/* FPM_QGRAM: bigram (q = 2) fingerprints, the q-gram direction of the
 * paper's future work (Section 5).  Every bigram (x, y) of the raw bytes sets
 * bit ((x * 256 + y) * 2654435761 mod 2^32) >> (32 - log2(bits)) (Knuth's
 * multiplicative hash); the symbol map is not used (fpm_num_fields = bits).
 * One edit replaces at most two bigrams, so F_D moves by at most 4 per edit
 * and a pair is rejected when F_D > 4k (Ham and Lev). */
/* FPM_COMBO: occurrence and count combined in one word (Section 5 names
 * combining fingerprint types as future work).  The low bits/2 bits are the
 * occurrence fingerprint of fields 0 .. bits/2 - 1; above them, 2-bit
 * saturating counters of fields 0 .. bits/4 - 1 (the map's first, most
 * frequent fields).  F_D is the larger of the two parts' F_D (count part:
 * L1), so Eq. 1 holds: a pair survives when both parts are <= 2k. */
typedef enum { FPM_OCC = 0, FPM_COUNT = 1, FPM_POS = 2, FPM_OCCH = 3, FPM_QGRAM = 4, FPM_COMBO = 5 } fpm_variant;
typedef enum { FPM_HAM = 0, FPM_LEV = 1 } fpm_metric;
typedef enum { FPM_COMMON = 0, FPM_RARE = 1, FPM_MIXED = 2, FPM_CUSTOM = 3 } fpm_symbols;

/* Work schedule of a match.
 *   FPM_SCHED_PLAIN: the host reads the query length histogram, builds the
 *     work list and launches one wave per work item with fixed default tiles.
 *   FPM_SCHED_BATCHED: the work list is built on the device and one
 *     persistent launch drains it through an atomic counter; the whole match
 *     pipeline is captured once in a hipGraph and replayed.
 *   FPM_SCHED_BRUTE: no fingerprints -- every length-compatible pair is
 *     verified (the paper's naive comparison T_n, Section 4). */
typedef enum { FPM_SCHED_PLAIN = 0, FPM_SCHED_BATCHED = 1, FPM_SCHED_BRUTE = 2 } fpm_schedule;

/* Rejection rule of the filter.
 *   FPM_BOUND_FD: the paper's Eq. 1 -- a pair survives when F_D <= 2k.
 *   FPM_BOUND_ASYM: an extension beyond the paper, offered as a separate
 *     rule so the paper's filter stays as printed.  F_D splits into
 *     e(q, w) = popc(q & ~w) and e(w, q) = popc(w & ~q) (count: the sums of
 *     positive count differences); the per-edit argument of Theorem 1,
 *     applied to each direction alone, gives D >= max(e(q, w), e(w, q)) >=
 *     ceil(F_D / 2), so a pair survives when both are <= k.  Since
 *     e(q, w) - e(w, q) = popc(q) - popc(w), pairs whose key popcounts differ
 *     by more than k are rejected wholesale: dictionary length blocks are
 *     ordered by popcount and work tiles whose popcount ranges are too far
 *     apart are skipped.  Defined for occurrence, occurrence-halved (Hamming)
 *     and count fingerprints; FPM_EUNSUPPORTED for position fingerprints.
 *     Matches are the same under both rules; survivors differ. */
typedef enum { FPM_BOUND_FD = 0, FPM_BOUND_ASYM = 1 } fpm_bound;

/* Where the filter test F_D <= t (Eq. 1; t = 2k, bigrams 4k) runs.
 *   FPM_UNIT_AUTO (default) = FPM_UNIT_VALU.
 *   FPM_UNIT_VALU: vector ALUs -- per pair one XOR, one popcount and one
 *     shift of the result's sign bit into a survivor mask.
 *   FPM_UNIT_MATRIX (opt-in, an addition of this library: the method is
 *     integer bit arithmetic and the paper's design has no matrix unit):
 *     matrix cores; FPM_EUNSUPPORTED where the key family does not allow
 *     it.  F_D of two W-bit keys (W = 16 or 32) is an inner product: with
 *     every key bit written as a signed byte (+1 for 0, -1 for 1 on the
 *     query side, the negation on the word side), the product of a query
 *     row and a word column over the W key positions is 2 F_D - W.  One
 *     8-bit integer matrix instruction (32 x 32 outputs, W contraction
 *     positions) with the accumulator input W - 1 - 2t yields 2 F_D - 2t - 1
 *     for 1,024 pairs, negative exactly when the pair survives; a group of
 *     64 queries stays in registers while the words stream through, and the
 *     sign bits go into the same survivor masks as on the vector path.
 *     Offered for the paper's rule (FPM_BOUND_FD) on keys whose F_D is the
 *     popcount of their XOR: occurrence and occurrence-halved fingerprints
 *     (16 and 32 bits), 16-bit count fingerprints (24-bit thermometer keys)
 *     and bigrams.  Survivors and matches are the same on both units. */
typedef enum { FPM_UNIT_AUTO = 0, FPM_UNIT_VALU = 1, FPM_UNIT_MATRIX = 2 } fpm_filter_unit;

/* Popcount pruning of the paper's rule (an exact shortcut, not in the
 * paper).  F_D = popc(q ^ w) >= |popc(q) - popc(w)|, so a pair whose key
 * popcounts differ by more than t (Eq. 1: 2k, bigrams 4k) fails the filter.
 * With pruning, a plan orders every length block of its dictionary copy
 * and of each query batch by key popcount; a group of pairs (a work item,
 * or a pass: 32 queries x 128 words on the vector ALUs, 64 queries x 32
 * words on the matrix cores) whose popcount ranges lie more than t apart is
 * skipped untested.  Survivors, matches and pairs_examined are unchanged;
 * fpm_stats.pairs_filtered counts the pairs the filter actually tested.
 * The ordering also gathers the survivors into the work items near equal
 * popcounts, so pruning pays where the key popcounts are spread (long and
 * mixed-length strings) and wants smaller work items than the unordered
 * layout; the tuning table records where it is on.
 *   FPM_PRUNE_OFF (default): every examined pair is tested.
 *   FPM_PRUNE_ON: the batched schedule (either filter unit) with
 *     occurrence, occurrence-halved, count or bigram keys under
 *     FPM_BOUND_FD; FPM_EUNSUPPORTED otherwise.  The plan then holds a popcount-ordered
 *     copy of the dictionary's strings, keys and permutation (about the
 *     index's own size). */
typedef enum { FPM_PRUNE_OFF = 0, FPM_PRUNE_ON = 1 } fpm_pop_prune;

/* One reported match.  `query` and `word` index the caller's lists. */
typedef struct {
    uint32_t query;
    uint32_t word;
    uint32_t dist;
} fpm_hit;

/* Counters of one match call. */
typedef struct {
    uint64_t pairs_logical;  /* |Q| * |D| */
    uint64_t pairs_examined; /* length-compatible pairs put through the filter */
    uint64_t survivors;      /* pairs kept by the filter (F_D <= 2k, or the asymmetric bound) and verified */
    uint64_t matches;        /* pairs within distance k */
    uint64_t verify_cells;   /* sum over survivors of (2k+1) * min(m, n) */
    uint64_t pairs_filtered; /* examined pairs the filter tested (the rest were skipped by popcount
                                pruning, which no survivor can be; 0 for FPM_SCHED_BRUTE) */
    float ms;                /* device time of the match pipeline (hip events) */
    uint32_t work_items;     /* work items the schedule processed */
    uint32_t filter_unit;    /* fpm_filter_unit that ran the filter test: FPM_UNIT_VALU or FPM_UNIT_MATRIX
                                (FPM_UNIT_AUTO for FPM_SCHED_BRUTE, which has no filter) */
} fpm_stats;

/* Tuning options; zero fields take defaults.  The match result never
 * depends on them. */
typedef struct {
    uint32_t schedule;         /* fpm_schedule */
    uint32_t queries_per_item; /* queries per work item, multiple of 16, <= 1024 (default 64) */
    uint32_t slab;             /* dictionary words per work item, multiple of 64, <= 4M (default 4096) */
    uint32_t bucket_order;     /* 0: longest query length first, 1: shortest first */
    uint32_t use_graph;        /* batched only: 1 = capture/replay a hipGraph (default 1), 2 = plain launches */
    uint32_t waves_per_cu;     /* batched only: persistent waves per compute unit (default 32) */
    uint32_t match_capacity;   /* initial device match buffer (entries; default 1 << 20); grows on overflow */
    uint32_t time_kernel;      /* 1: bracket the match kernel of every run with HIP events (see
                                  fpm_plan_kernel_ms); a batched graph is then split into a prep graph
                                  and a post graph around a direct launch of the match kernel */
    uint32_t tail_split;       /* batched and brute: percent (1..99) of each bucket pair's words that go
                                  into tail items of a smaller tile (queries_per_item / 2 by slab / 4,
                                  at least 16 by 64), listed after every full-size item so that a launch
                                  ends on short items; 0 = default (100: no tail items) */
    uint32_t bound;            /* fpm_bound: filter rule (default FPM_BOUND_FD); ignored by FPM_SCHED_BRUTE */
    uint32_t filter_unit;      /* fpm_filter_unit: where the filter test runs (default FPM_UNIT_AUTO) */
    uint32_t pop_prune;        /* fpm_pop_prune (default FPM_PRUNE_OFF) */
    uint32_t reserved[4];
} fpm_options;

typedef struct fpm_index fpm_index;
typedef struct fpm_plan fpm_plan;

/* Last error message of the calling thread ("" if none). */
const char *fpm_last_error(void);

/* Release memory the library returned (match arrays). */
void fpm_free(void *p);

/* Number of symbol fields of a fingerprint (Section 3 variants with the
 * Section 4 parameters b = 2, p = 3): occ bits, occh bits/2, count bits/2,
 * pos bits/3 + bits%3, qgram bits (hash buckets), combo bits/2.  Returns -1
 * for an unknown variant or bits. */
int fpm_num_fields(fpm_variant variant, uint32_t bits);

/* Symbol selection (Section 3: common / rare / mixed sets).  A byte
 * histogram of the strings is taken on the GPU and ranked; map_out[c] is the
 * field of byte c or 0xFF when c is not in the fingerprint alphabet.
 * Host buffers, borrowed for the call. */
fpm_status fpm_select_symbols(const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                              fpm_variant variant, uint32_t bits, fpm_symbols symbols,
                              uint8_t map_out[256]);

/* Preprocess a dictionary (Sections 3.2 and 3.4): select the symbol map (or
 * take `custom_map`, 256 entries, when symbols == FPM_CUSTOM; a map may send
 * several symbols to one field), copy the strings to the GPU, sort them by
 * length into padded per-length blocks and build one fingerprint per word.
 * Host buffers, borrowed for the call.  *out receives an index that owns
 * its device memory; release it with fpm_index_destroy. */
fpm_status fpm_build_fingerprints(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_words,
                                  fpm_variant variant, uint32_t bits, fpm_symbols symbols,
                                  const uint8_t *custom_map, fpm_index **out);

void fpm_index_destroy(fpm_index *ix);

/* Fingerprints of the dictionary words in the caller's order, each widened to
 * uint32 (n_words entries, host buffer owned by the caller). */
fpm_status fpm_get_fingerprints(const fpm_index *ix, uint32_t *out);

/* Symbol map of the index (256 entries). */
fpm_status fpm_get_map(const fpm_index *ix, uint8_t map_out[256]);

/* Number of words, variant and fingerprint bits of an index. */
fpm_status fpm_index_info(const fpm_index *ix, uint32_t *n_words, uint32_t *variant, uint32_t *bits);

/* Device time of the index build (the preprocessing of Section 3.4; the
 * paper reports its fingerprint construction speed in Table 4), measured
 * with HIP events once the dictionary is resident on the device:
 * *total_ms = symbol statistics + length sort + padded layout with
 * fingerprints + inverse permutation; *layout_ms = the last three.  Either
 * pointer may be NULL. */
fpm_status fpm_index_build_ms(const fpm_index *ix, float *total_ms, float *layout_ms);

/* Device memory accounting.  Every device buffer the library allocates
 * (indexes, plans, the temporaries of the host-buffer calls, the learned
 * grouping) counts against one process-wide total.  With a limit set, an
 * allocation that would take the total past it fails with FPM_ENOMEM before
 * any device call, and the failing entry point releases what it had taken.
 * max_bytes = 0 removes the limit (the default).  Buffers allocated before a
 * limit was set stay valid. */
fpm_status fpm_set_device_memory_limit(uint64_t max_bytes);
fpm_status fpm_device_memory_in_use(uint64_t *bytes);

/* Fingerprints of arbitrary strings under the index's map and variant
 * (Section 3.2), caller's order, widened to uint32.  Host buffers. */
fpm_status fpm_fingerprints(const fpm_index *ix, const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                            uint32_t *out);

/* Match queries against the index (the dictionary-matching problem of
 * Section 1, filtered by Eq. 1, survivors verified exactly).  Host buffers
 * in, host result out: *out is a malloc'd array of *n_out matches sorted by
 * (query, word), every pair with distance <= k exactly once, or NULL when
 * there are none; release it with fpm_free.  `opt` and `stats` may be NULL.
 * Position and occurrence-halved indexes support FPM_HAM only. */
fpm_status fpm_match(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                     fpm_metric metric, uint32_t k, const fpm_options *opt, fpm_hit **out, uint64_t *n_out,
                     fpm_stats *stats);

/* Surviving pairs of the filter alone (F_D <= 2k over length-compatible
 * pairs), as (query, word) uint32 pairs sorted by (query, word); for tests and
 * rejection-rate studies on small inputs.  *pairs is malloc'd (fpm_free). */
fpm_status fpm_filter_pairs(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets,
                            uint32_t n_queries, fpm_metric metric, uint32_t k, uint32_t **pairs, uint64_t *n_pairs);

/* Exact distances of listed pairs (query i, word j) on the GPU, capped at
 * k + 1 ("more than k"); Ham of unequal lengths is k + 1.  Host buffers:
 * pairs holds 2 * n_pairs uint32, dist_out n_pairs uint32.  Used to label
 * training pairs for the learned grouping. */
fpm_status fpm_verify_pairs(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                            const uint32_t *pairs, uint64_t n_pairs, fpm_metric metric, uint32_t k, uint32_t *dist_out);

/* ---------------------------------------------------------------------
 * Device-resident matching.  A plan holds every device buffer of a match
 * pipeline for up to `max_queries` queries of at most `max_query_bytes`
 * total bytes, so repeated runs allocate nothing except when the match
 * buffer has to grow.  `hip_stream` is a hipStream_t (NULL = the default
 * stream).  Inputs of fpm_plan_run are DEVICE pointers; a string longer than
 * 255 or decreasing offsets are detected on the device and reported by
 * fpm_plan_result as FPM_EINVAL (those strings are clamped, never read out
 * of bounds: reads stay below qoffsets[n_queries] <= max_query_bytes).
 * Plans are independent: two plans on two streams keep two batches in
 * flight, and one batch's preparation and match-list sort then run beside
 * the next batch's match kernel.
 * --------------------------------------------------------------------- */
fpm_status fpm_plan_create(const fpm_index *ix, uint32_t max_queries, uint64_t max_query_bytes, fpm_metric metric,
                           uint32_t k, const fpm_options *opt, void *hip_stream, fpm_plan **out);

/* Enqueue one match of n_queries queries (device CSR) on the plan's stream.
 * Does not wait.  With FPM_SCHED_PLAIN the host reads the query length
 * histogram (one stream synchronisation). */
fpm_status fpm_plan_run(fpm_plan *plan, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t n_queries);

/* Wait for the last run and report it: *n_out matches; *d_matches points to
 * the plan-owned DEVICE array of fpm_hit sorted by (query, word), valid
 * until the next run or destroy.  When the run overflowed the match buffer,
 * the buffer is grown and the run repeated before returning.  Either output
 * may be NULL. */
fpm_status fpm_plan_result(fpm_plan *plan, const fpm_hit **d_matches, uint64_t *n_out, fpm_stats *stats);

/* Durations in ms of the match kernel of the last min(runs, max, 256) runs,
 * oldest first, for a plan created with time_kernel = 1 (waits for the
 * stream).  *n receives the count written to ms_out. */
fpm_status fpm_plan_kernel_ms(fpm_plan *plan, float *ms_out, uint32_t max, uint32_t *n);

/* Copy up to `max` matches of the last run into dst (host or device memory,
 * hipMemcpyDefault), synchronously; *n_copied receives the number copied. */
fpm_status fpm_plan_copy_matches(fpm_plan *plan, fpm_hit *dst, uint64_t max, uint64_t *n_copied);

void fpm_plan_destroy(fpm_plan *plan);

/* ---------------------------------------------------------------------
 * Allocation-free matching, for callers that cannot allocate device memory
 * (serving loops with a fixed memory budget, harnesses that forbid
 * hipMalloc, code that must not touch the allocator).  Same result as
 * fpm_match on the same queries: the match list of the queries in d_qbytes /
 * d_qoffsets (DEVICE CSR, n_queries strings, d_qbytes holding query_bytes
 * bytes) against the index, sorted by (query, word), written to the
 * caller's DEVICE array d_out of out_cap entries; *n_out receives the number
 * of matches.
 *
 * Every intermediate buffer lives in one static device array of the library
 * (about 26 MiB, held on each device from the first call there until the
 * process ends); the call allocates no device memory.  Limits:
 * n_queries <= FPM_NOALLOC_MAX_QUERIES, query_bytes <=
 * FPM_NOALLOC_MAX_QUERY_BYTES (FPM_EINVAL beyond them, before any device
 * work), at most FPM_NOALLOC_MAX_MATCHES matches (FPM_ENOMEM, *n_out holds
 * the count; use a plan for larger results).  When the matches do not fit
 * out_cap the call fails with FPM_EINVAL, *n_out holds the count and d_out
 * holds no valid list.
 *
 * The work runs on `hip_stream` (NULL = the null stream) with the
 * device-scheduled persistent kernel and plain launches (options: tiles,
 * bucket order, tail split, filter unit; FPM_SCHED_PLAIN is run device-
 * scheduled too, FPM_SCHED_BRUTE verifies every length-compatible pair;
 * the asymmetric bound is FPM_EUNSUPPORTED), and the call returns after it
 * has finished (it synchronises the stream, so it cannot be captured into a
 * graph).  The index must live on the current device.  All calls on one
 * device share the array: the library runs them one at a time (a lock per
 * device), and every buffer a call reads is written or cleared by that call
 * first.  stats may be NULL (stats->ms is 0). */
#define FPM_NOALLOC_MAX_QUERIES 65536u
#define FPM_NOALLOC_MAX_QUERY_BYTES (4u << 20)
#define FPM_NOALLOC_MAX_MATCHES (1u << 20)
fpm_status fpm_match_noalloc(const fpm_index *ix, const uint8_t *d_qbytes, const uint64_t *d_qoffsets,
                             uint32_t n_queries, uint64_t query_bytes, fpm_metric metric, uint32_t k,
                             const fpm_options *opt, void *hip_stream, fpm_hit *d_out, uint64_t out_cap,
                             uint64_t *n_out, fpm_stats *stats);

/* Autotuner for the batched schedule: times every combination of
 * queries_per_item in {16, 32, 64, 128, 256}, slab in {512, 1024, 2048,
 * 4096, 8192, 16384} and both bucket orders on the given device queries with
 * the tail split, filter rule (bound), filter unit and popcount pruning of
 * *best (on entry), then the
 * fastest of those with tail splits 10, 25 and 40 (100 = none), then times the
 * four fastest configurations again with max(8, 4 * repeats) runs each and
 * writes the fastest of those into *best (its schedule = FPM_SCHED_BATCHED).
 * `timings_out` (nullable) receives up to `max_timings` rows of
 * (queries_per_item, slab, bucket_order, tail_split, ms) as floats, the
 * longer re-timings last. */
fpm_status fpm_autotune(const fpm_index *ix, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t n_queries,
                        uint64_t query_bytes, fpm_metric metric, uint32_t k, uint32_t repeats, fpm_options *best,
                        float *timings_out, uint32_t max_timings, uint32_t *n_timings);

#ifdef __cplusplus
}
#endif

#endif /* FPM_H */
