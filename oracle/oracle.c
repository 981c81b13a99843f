/*
 * oracle.c -- CPU oracle for fingerprint-filtered approximate dictionary
 * matching (Cislak & Grabowski, "Lightweight Fingerprints for Fast Approximate
 * Keyword Matching Using Bitwise Operations", arXiv:1711.08475).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * reads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Everything here is written to be slow and obviously correct:
 *   - Hamming distance: full mismatch count, "infinite" when lengths differ
 *     (Section 1 definition; proof of Theorem 1).
 *   - Levenshtein distance: the full (m+1) x (n+1) Wagner-Fischer table
 *     (Section 1 definition: unit-cost insertions, deletions, substitutions).
 *   - Brute-force matching: every (query, word) pair, no fingerprints, no
 *     length pruning unless the caller asks for the separately labelled
 *     length-pruned mode (which relies on Lev >= |m-n| and Ham = inf for m!=n).
 *   - Fingerprints built by the construction steps of Section 3.2, compared
 *     by the distances of Section 3.3 (Eq. 1 threshold 2k).
 *
 * Readings of the paper used here (each is also listed in the design notes):
 *   - Field j of the symbol map sits at the j-th least significant bits
 *     (occ: bit j; count: bits 2j..2j+1; pos: bits 3j..3j+2, occurrence bits
 *     after the position fields; occ-halved: bit 2j first half, 2j+1 second
 *     half).  The paper prints rank 0 leftmost; the integer layout puts it in
 *     the least significant bit.  F_D does not depend on this layout.
 *   - Count distance: the paper's Hamming weight of the XOR of binary
 *     saturating counters is unsound (the strings "eet" and "ett" are one
 *     substitution apart but their 2-bit counters differ in 4 bits), so the
 *     filter distance is the L1 distance of the saturated counts.  The
 *     literal XOR weight is kept as a diagnostic only.
 *   - Position distance: number of mismatching p-bit position fields plus the
 *     Hamming weight of the XOR of the trailing occurrence bits.
 *   - A symbol map may be many-to-one (several symbols share one field); the
 *     constructions then act on the union of those symbols.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_HAM 0
#define ORC_LEV 1

#define ORC_OCC 0
#define ORC_COUNT 1
#define ORC_POS 2
#define ORC_OCCH 3
#define ORC_QGRAM 4  /* hashed bigram occurrence (q = 2); future work of Section 5 */
#define ORC_COMBO 5  /* occurrence and count in one word; future work of Section 5 */

#define ORC_COMMON 0
#define ORC_RARE 1
#define ORC_MIXED 2

#define ORC_NONE 0xFFu   /* symbol not in the fingerprint alphabet */
#define ORC_INF 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Distances (Section 1)                                                     */
/* ------------------------------------------------------------------------ */

/* Hamming distance: number of positions with different symbols; infinite
 * (ORC_INF) when the two lengths differ. */
uint32_t orc_ham(const uint8_t *a, uint32_t m, const uint8_t *b, uint32_t n)
{
    if (m != n)
        return ORC_INF;
    uint32_t d = 0;
    for (uint32_t i = 0; i < m; ++i)
        if (a[i] != b[i])
            d++;
    return d;
}

/* Levenshtein distance: the full Wagner-Fischer table
 *   D[i][0] = i, D[0][j] = j,
 *   D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a_i != b_j]).
 * `table` must hold (m+1)*(n+1) cells. */
static uint32_t lev_table(const uint8_t *a, uint32_t m, const uint8_t *b, uint32_t n, uint32_t *table)
{
    const uint32_t w = n + 1;
    for (uint32_t i = 0; i <= m; ++i)
        table[i * w + 0] = i;
    for (uint32_t j = 0; j <= n; ++j)
        table[0 * w + j] = j;
    for (uint32_t i = 1; i <= m; ++i) {
        for (uint32_t j = 1; j <= n; ++j) {
            uint32_t del = table[(i - 1) * w + j] + 1;
            uint32_t ins = table[i * w + (j - 1)] + 1;
            uint32_t sub = table[(i - 1) * w + (j - 1)] + (a[i - 1] != b[j - 1] ? 1u : 0u);
            uint32_t best = del < ins ? del : ins;
            table[i * w + j] = best < sub ? best : sub;
        }
    }
    return table[m * w + n];
}

uint32_t orc_lev(const uint8_t *a, uint32_t m, const uint8_t *b, uint32_t n)
{
    uint32_t *table = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m + 1) * (n + 1));
    if (!table)
        return ORC_INF;
    uint32_t d = lev_table(a, m, b, n, table);
    free(table);
    return d;
}

/* ------------------------------------------------------------------------ */
/* Brute-force dictionary matching (Section 1 problem statement)            */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t *v; /* triples (query, word, dist) */
    uint64_t n, cap;
} triples;

static int push(triples *t, uint32_t q, uint32_t w, uint32_t d)
{
    if (t->n == t->cap) {
        uint64_t nc = t->cap ? t->cap * 2 : 1024;
        uint32_t *nv = (uint32_t *)realloc(t->v, sizeof(uint32_t) * 3 * nc);
        if (!nv)
            return -1;
        t->v = nv;
        t->cap = nc;
    }
    t->v[3 * t->n + 0] = q;
    t->v[3 * t->n + 1] = w;
    t->v[3 * t->n + 2] = d;
    t->n++;
    return 0;
}

typedef struct {
    const uint8_t *dbytes;
    const uint64_t *doffs;
    uint32_t nd;
    const uint8_t *qbytes;
    const uint64_t *qoffs;
    uint32_t nq;
    int metric;
    uint32_t k;
    int length_pruned;
    volatile uint32_t next_query; /* shared work counter */
    int failed;
} match_job;

typedef struct {
    match_job *job;
    triples out;
} match_worker;

static void *match_thread(void *arg)
{
    match_worker *wk = (match_worker *)arg;
    match_job *job = wk->job;
    uint32_t *table = (uint32_t *)malloc(sizeof(uint32_t) * 256u * 256u);
    if (!table) {
        job->failed = 1;
        return NULL;
    }
    for (;;) {
        uint32_t q = __sync_fetch_and_add(&job->next_query, 1u);
        if (q >= job->nq)
            break;
        const uint8_t *a = job->qbytes + job->qoffs[q];
        uint32_t m = (uint32_t)(job->qoffs[q + 1] - job->qoffs[q]);
        for (uint32_t w = 0; w < job->nd; ++w) {
            const uint8_t *b = job->dbytes + job->doffs[w];
            uint32_t n = (uint32_t)(job->doffs[w + 1] - job->doffs[w]);
            uint32_t d;
            if (job->metric == ORC_HAM) {
                d = orc_ham(a, m, b, n);
            } else {
                if (job->length_pruned && (m > n ? m - n : n - m) > job->k)
                    continue; /* labelled mode: Lev >= |m - n| > k */
                d = lev_table(a, m, b, n, table);
            }
            if (d != ORC_INF && d <= job->k) {
                if (push(&wk->out, q, w, d)) {
                    job->failed = 1;
                    free(table);
                    return NULL;
                }
            }
        }
    }
    free(table);
    return NULL;
}

static int cmp_triple(const void *x, const void *y)
{
    const uint32_t *a = (const uint32_t *)x, *b = (const uint32_t *)y;
    if (a[0] != b[0])
        return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1])
        return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* Number of host threads this process may run on. */
uint32_t orc_host_threads(void)
{
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0)
            return (uint32_t)c;
    }
    return 1;
}

/* All (query, word, dist) with dist <= k, sorted by (query, word).
 * Strings longer than 255 are rejected (-1).  The result array (3 uint32 per
 * match) is malloc'd; release it with orc_free.  Returns 0 on success. */
int orc_match(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd,
              const uint8_t *qbytes, const uint64_t *qoffs, uint32_t nq,
              int metric, uint32_t k, uint32_t nthreads, int length_pruned,
              uint32_t **out, uint64_t *n_out)
{
    *out = NULL;
    *n_out = 0;
    if (metric != ORC_HAM && metric != ORC_LEV)
        return -1;
    for (uint32_t i = 0; i < nd; ++i)
        if (doffs[i + 1] < doffs[i] || doffs[i + 1] - doffs[i] > 255)
            return -1;
    for (uint32_t i = 0; i < nq; ++i)
        if (qoffs[i + 1] < qoffs[i] || qoffs[i + 1] - qoffs[i] > 255)
            return -1;
    if (nthreads == 0)
        nthreads = orc_host_threads();
    match_job job;
    memset(&job, 0, sizeof(job));
    job.dbytes = dbytes;
    job.doffs = doffs;
    job.nd = nd;
    job.qbytes = qbytes;
    job.qoffs = qoffs;
    job.nq = nq;
    job.metric = metric;
    job.k = k;
    job.length_pruned = length_pruned;
    match_worker *wk = (match_worker *)calloc(nthreads, sizeof(match_worker));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    if (!wk || !th) {
        free(wk);
        free(th);
        return -1;
    }
    for (uint32_t t = 0; t < nthreads; ++t) {
        wk[t].job = &job;
        pthread_create(&th[t], NULL, match_thread, &wk[t]);
    }
    uint64_t total = 0;
    for (uint32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        total += wk[t].out.n;
    }
    int rc = job.failed ? -1 : 0;
    uint32_t *all = NULL;
    if (rc == 0 && total) {
        all = (uint32_t *)malloc(sizeof(uint32_t) * 3 * total);
        if (!all)
            rc = -1;
    }
    uint64_t pos = 0;
    for (uint32_t t = 0; t < nthreads; ++t) {
        if (rc == 0 && wk[t].out.n) {
            memcpy(all + 3 * pos, wk[t].out.v, sizeof(uint32_t) * 3 * wk[t].out.n);
            pos += wk[t].out.n;
        }
        free(wk[t].out.v);
    }
    free(wk);
    free(th);
    if (rc)
        return rc;
    if (total)
        qsort(all, total, sizeof(uint32_t) * 3, cmp_triple);
    *out = all;
    *n_out = total;
    return 0;
}

/* Exact distance of explicitly listed pairs (query i against word j).
 * dist[p] = ORC_INF for an infinite Hamming distance. */
int orc_pair_dist(const uint8_t *dbytes, const uint64_t *doffs, const uint8_t *qbytes,
                  const uint64_t *qoffs, const uint32_t *pairs, uint64_t npairs,
                  int metric, uint32_t *dist)
{
    uint32_t *table = (uint32_t *)malloc(sizeof(uint32_t) * 256u * 256u);
    if (!table)
        return -1;
    for (uint64_t p = 0; p < npairs; ++p) {
        uint32_t q = pairs[2 * p], w = pairs[2 * p + 1];
        const uint8_t *a = qbytes + qoffs[q];
        uint32_t m = (uint32_t)(qoffs[q + 1] - qoffs[q]);
        const uint8_t *b = dbytes + doffs[w];
        uint32_t n = (uint32_t)(doffs[w + 1] - doffs[w]);
        if (m > 255 || n > 255) {
            free(table);
            return -1;
        }
        dist[p] = metric == ORC_HAM ? orc_ham(a, m, b, n) : lev_table(a, m, b, n, table);
    }
    free(table);
    return 0;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Fingerprint alphabet (Section 3: common / rare / mixed symbol sets)       */
/* ------------------------------------------------------------------------ */

/* Number of symbol fields a fingerprint of `bits` bits holds (Section 3 list
 * of variants, parameters of Section 4: b = 2 bits per count, p = 3 bits per
 * position, the leftover bits of the position variant are occurrence bits). */
int orc_num_fields(int variant, uint32_t bits)
{
    if (bits != 16 && bits != 32)
        return -1;
    switch (variant) {
    case ORC_OCC:
        return (int)bits;
    case ORC_OCCH:
        return (int)bits / 2;
    case ORC_COUNT:
        return (int)bits / 2;
    case ORC_POS:
        return (int)(bits / 3) + (int)(bits % 3);
    case ORC_QGRAM:
        return (int)bits; /* fields are hash buckets; the symbol map is not used */
    case ORC_COMBO:
        return (int)bits / 2; /* occurrence fields; the first bits/4 also have counters */
    default:
        return -1;
    }
}

/* Number of p-bit position fields of the position variant. */
static int pos_fields(uint32_t bits) { return (int)(bits / 3); }

/* Total occurrences of each byte value over all strings. */
void orc_histogram(const uint8_t *bytes, const uint64_t *offs, uint32_t n, uint64_t hist[256])
{
    memset(hist, 0, sizeof(uint64_t) * 256);
    for (uint32_t i = 0; i < n; ++i)
        for (uint64_t t = offs[i]; t < offs[i + 1]; ++t)
            hist[bytes[t]]++;
}

/* Build the symbol -> field map from a byte histogram.
 * Symbols are ranked by total occurrences, most frequent first, ties by byte
 * value ascending; only symbols that occur are eligible.
 *   common: the F most frequent symbols, in that order;
 *   rare:   the F least frequent symbols, least frequent first;
 *   mixed:  the ceil(F/2) most frequent, then the floor(F/2) least frequent
 *           (a symbol already taken is skipped).
 * The i-th selected symbol gets field i.  Returns the number of symbols
 * mapped, or -1 on bad arguments. */
int orc_select_symbols(const uint64_t hist[256], int variant, uint32_t bits, int symset, uint8_t map[256])
{
    int nf = orc_num_fields(variant, bits);
    if (nf < 0 || symset < ORC_COMMON || symset > ORC_MIXED)
        return -1;
    /* descending-frequency order of the present symbols (selection sort,
     * plain on purpose) */
    int order[256], present = 0;
    int used[256];
    memset(used, 0, sizeof(used));
    for (;;) {
        int best = -1;
        for (int c = 0; c < 256; ++c) {
            if (used[c] || hist[c] == 0)
                continue;
            if (best < 0 || hist[c] > hist[best])
                best = c; /* strict '>' keeps the smaller byte on ties */
        }
        if (best < 0)
            break;
        used[best] = 1;
        order[present++] = best;
    }
    /* ascending-frequency order: least frequent first, ties by byte
     * ascending */
    int rorder[256], rn = 0;
    memset(used, 0, sizeof(used));
    for (;;) {
        int best = -1;
        for (int c = 0; c < 256; ++c) {
            if (used[c] || hist[c] == 0)
                continue;
            if (best < 0 || hist[c] < hist[best])
                best = c;
        }
        if (best < 0)
            break;
        used[best] = 1;
        rorder[rn++] = best;
    }
    int chosen[256], nc = 0;
    int taken[256];
    memset(taken, 0, sizeof(taken));
    if (symset == ORC_COMMON) {
        for (int i = 0; i < present && nc < nf; ++i)
            chosen[nc++] = order[i];
    } else if (symset == ORC_RARE) {
        for (int i = 0; i < rn && nc < nf; ++i)
            chosen[nc++] = rorder[i];
    } else {
        int half_common = (nf + 1) / 2;
        for (int i = 0; i < present && nc < half_common; ++i) {
            chosen[nc++] = order[i];
            taken[order[i]] = 1;
        }
        for (int i = 0; i < rn && nc < nf; ++i) {
            if (taken[rorder[i]])
                continue;
            chosen[nc++] = rorder[i];
            taken[rorder[i]] = 1;
        }
    }
    memset(map, ORC_NONE, 256);
    for (int i = 0; i < nc; ++i)
        map[chosen[i]] = (uint8_t)i;
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Fingerprint construction (Section 3.2)                                    */
/* ------------------------------------------------------------------------ */

/* occurrence: iterate the string; for each mapped symbol shift 0x1 left by
 * its field index and OR it in. */
static uint32_t fp_occ(const uint8_t *s, uint32_t n, const uint8_t *map)
{
    uint32_t fp = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint8_t q = map[s[i]];
        if (q != ORC_NONE)
            fp |= 1u << q;
    }
    return fp;
}

/* occurrence halved: occurrences in S[1..floor(n/2)] and S[floor(n/2)+1..n];
 * field j uses bit 2j for the first half and bit 2j+1 for the second half. */
static uint32_t fp_occh(const uint8_t *s, uint32_t n, const uint8_t *map)
{
    uint32_t fp = 0, half = n / 2;
    for (uint32_t i = 0; i < half; ++i) {
        uint8_t q = map[s[i]];
        if (q != ORC_NONE)
            fp |= 1u << (2u * q);
    }
    for (uint32_t i = half; i < n; ++i) {
        uint8_t q = map[s[i]];
        if (q != ORC_NONE)
            fp |= 1u << (2u * q + 1u);
    }
    return fp;
}

/* count (b = 2): per mapped symbol, increment the 2-bit counter at bits
 * q, q+1 (q = 2 * field) the way the paper describes it: a clear right
 * (low) bit is set; a set right bit with a set left bit means the counter
 * is saturated at 3 and stays; a set right bit with a clear left bit
 * becomes left set, right clear (1 -> 2). */
static uint32_t fp_count(const uint8_t *s, uint32_t n, const uint8_t *map)
{
    uint32_t fp = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint8_t f = map[s[i]];
        if (f == ORC_NONE)
            continue;
        uint32_t q = 2u * f;
        uint32_t right = 1u << q, left = 1u << (q + 1u);
        if (!(fp & right)) {
            fp |= right;
        } else if (fp & left) {
            /* already 3: saturated */
        } else {
            fp |= left;
            fp &= ~right;
        }
    }
    return fp;
}

/* position (p = 3): for each position field j, the 0-indexed first position
 * of a symbol mapped to j, written as all ones (2^p - 1) when that position is
 * >= 2^p - 1 or when no such symbol occurs; the remaining fields are single
 * occurrence bits placed after the position fields. */
static uint32_t fp_pos(const uint8_t *s, uint32_t n, const uint8_t *map, uint32_t bits)
{
    const uint32_t p = 3, allones = (1u << p) - 1u;
    int npos = pos_fields(bits);
    int nf = orc_num_fields(ORC_POS, bits);
    uint32_t fp = 0;
    for (int j = 0; j < npos; ++j) {
        uint32_t first = allones;
        for (uint32_t i = 0; i < n; ++i) {
            if (map[s[i]] == (uint8_t)j) {
                first = i;
                break;
            }
        }
        if (first >= allones)
            first = allones;
        fp |= first << (p * (uint32_t)j);
    }
    for (int j = npos; j < nf; ++j) {
        for (uint32_t i = 0; i < n; ++i) {
            if (map[s[i]] == (uint8_t)j) {
                fp |= 1u << (p * (uint32_t)npos + (uint32_t)(j - npos));
                break;
            }
        }
    }
    return fp;
}

/* q-gram occurrence (q = 2), an extension in the direction the paper names
 * as future work (Section 5): every bigram (s[i], s[i+1]) of the raw bytes
 * goes to one of the `bits` fields by Knuth's multiplicative hash of the
 * 16-bit value v = s[i] * 256 + s[i+1]: field = (v * 2654435761 mod 2^32)
 * >> (32 - log2(bits)); the field's bit is set.  Strings shorter than 2
 * have no bigram (fingerprint 0). */
static uint32_t fp_qgram(const uint8_t *s, uint32_t n, uint32_t bits)
{
    uint32_t lg = 0;
    while ((1u << lg) < bits)
        lg++;
    uint32_t fp = 0;
    for (uint32_t i = 0; i + 1 < n; ++i) {
        uint32_t v = (uint32_t)s[i] * 256u + (uint32_t)s[i + 1];
        uint32_t h = (uint32_t)((uint64_t)v * 2654435761ull % 4294967296ull);
        fp |= 1u << (h >> (32 - lg));
    }
    return fp;
}

/* Combined occurrence + count (Section 5 names combining fingerprint types
 * as future work): the low bits/2 bits are the occurrence fingerprint of
 * fields 0 .. bits/2 - 1; above them, the count fingerprint (2-bit saturating
 * counters) of fields 0 .. bits/4 - 1 -- the map's first, most frequent
 * fields get both. */
static uint32_t fp_combo(const uint8_t *s, uint32_t n, const uint8_t *map, uint32_t bits)
{
    uint8_t cmap[256];
    for (int c = 0; c < 256; ++c)
        cmap[c] = (map[c] != ORC_NONE && map[c] < bits / 4) ? map[c] : (uint8_t)ORC_NONE;
    return fp_occ(s, n, map) | (fp_count(s, n, cmap) << (bits / 2));
}

/* Fingerprint of one string.  Map entries must be < orc_num_fields or
 * ORC_NONE (checked by orc_check_map). */
uint32_t orc_fp(const uint8_t *s, uint32_t n, int variant, uint32_t bits, const uint8_t *map)
{
    switch (variant) {
    case ORC_OCC:
        return fp_occ(s, n, map);
    case ORC_OCCH:
        return fp_occh(s, n, map);
    case ORC_COUNT:
        return fp_count(s, n, map);
    case ORC_POS:
        return fp_pos(s, n, map, bits);
    case ORC_QGRAM:
        return fp_qgram(s, n, bits);
    case ORC_COMBO:
        return fp_combo(s, n, map, bits);
    default:
        return 0;
    }
}

int orc_check_map(const uint8_t *map, int variant, uint32_t bits)
{
    int nf = orc_num_fields(variant, bits);
    if (nf < 0)
        return -1;
    for (int c = 0; c < 256; ++c)
        if (map[c] != ORC_NONE && map[c] >= nf)
            return -1;
    return 0;
}

/* Fingerprints of a CSR string list. */
int orc_fp_many(const uint8_t *bytes, const uint64_t *offs, uint32_t n, int variant, uint32_t bits,
                const uint8_t *map, uint32_t *out)
{
    if (orc_check_map(map, variant, bits))
        return -1;
    for (uint32_t i = 0; i < n; ++i)
        out[i] = orc_fp(bytes + offs[i], (uint32_t)(offs[i + 1] - offs[i]), variant, bits, map);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fingerprint distance (Section 3.3) and the rejection rule (Eq. 1)        */
/* ------------------------------------------------------------------------ */

static uint32_t popcount32(uint32_t x)
{
    uint32_t c = 0;
    while (x) {
        c += x & 1u;
        x >>= 1;
    }
    return c;
}

/* F_D of two fingerprints.
 *   occ, occ-halved, q-gram: Hamming weight of the XOR;
 *   combined: the larger of the occurrence part's and the count part's F_D;
 *   count: L1 distance of the 2-bit saturated counts (sound reading);
 *          with literal != 0: the Hamming weight of the XOR as printed;
 *   pos:   number of position fields that differ + Hamming weight of the XOR
 *          of the occurrence bits. */
uint32_t orc_fd(uint32_t a, uint32_t b, int variant, uint32_t bits, int literal)
{
    switch (variant) {
    case ORC_OCC:
    case ORC_OCCH:
    case ORC_QGRAM:
        return popcount32(a ^ b);
    case ORC_COUNT: {
        if (literal)
            return popcount32(a ^ b);
        uint32_t d = 0;
        for (uint32_t j = 0; j < bits / 2; ++j) {
            int ca = (int)((a >> (2 * j)) & 3u), cb = (int)((b >> (2 * j)) & 3u);
            d += (uint32_t)(ca > cb ? ca - cb : cb - ca);
        }
        return d;
    }
    case ORC_COMBO: {
        /* each part is a sound F_D of its own (Theorem 1), so their maximum
         * is one too: a pair survives when both parts are <= 2k */
        uint32_t half = bits / 2, mask = (1u << half) - 1u;
        uint32_t occ = popcount32((a ^ b) & mask);
        uint32_t cnt = orc_fd(a >> half, b >> half, ORC_COUNT, half, 0);
        return occ > cnt ? occ : cnt;
    }
    case ORC_POS: {
        uint32_t d = 0;
        int npos = pos_fields(bits);
        for (int j = 0; j < npos; ++j)
            if (((a >> (3 * j)) & 7u) != ((b >> (3 * j)) & 7u))
                d++;
        uint32_t occ_part = (a ^ b) >> (3 * npos);
        return d + popcount32(occ_part);
    }
    default:
        return ORC_INF;
    }
}

/* Excess of fingerprint a over fingerprint b -- the one-directional half
 * of F_D used by the asymmetric bound (an extension beyond the paper's
 * Eq. 1, not one of its filters):
 *   occ, occ-halved: number of fields set in a and clear in b;
 *   count: sum over fields of max(c_a - c_b, 0) of the saturated counts;
 *   pos: not defined (ORC_INF).
 * excess(a, b) + excess(b, a) = F_D.  One edit changes each direction's
 * excess by at most one (a field can only gain or lose one unit), so the
 * distance is at least max(excess(a, b), excess(b, a)), which is itself at
 * least ceil(F_D / 2): a pair can be rejected when either excess exceeds k.
 * (For occ-halved this holds for Hamming only, as F_D itself does.) */
uint32_t orc_excess(uint32_t a, uint32_t b, int variant, uint32_t bits)
{
    switch (variant) {
    case ORC_OCC:
    case ORC_OCCH:
        return popcount32(a & ~b);
    case ORC_COUNT: {
        uint32_t d = 0;
        for (uint32_t j = 0; j < bits / 2; ++j) {
            int ca = (int)((a >> (2 * j)) & 3u), cb = (int)((b >> (2 * j)) & 3u);
            if (ca > cb)
                d += (uint32_t)(ca - cb);
        }
        return d;
    }
    default:
        return ORC_INF;
    }
}

void orc_excess_many(const uint32_t *a, const uint32_t *b, uint64_t n, int variant, uint32_t bits, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = orc_excess(a[i], b[i], variant, bits);
}

/* Largest F_D a pair within distance k can have: 2k (Eq. 1: one edit moves
 * F_D by at most 2, Theorems 1 and 2); for bigram fingerprints 4k (one edit
 * removes at most two bigram occurrences and adds at most two, so F_D moves
 * by at most 4). */
uint32_t orc_threshold(int variant, uint32_t k) { return variant == ORC_QGRAM ? 4 * k : 2 * k; }

/* Filter statistics over all (query, word) pairs.  A pair is examined when
 * it can match at all by length (Ham: equal lengths; Lev: |m-n| <= k); it
 * survives when ceil(F_D/2) <= k, i.e. F_D <= 2k (Eq. 1).  counts[0] =
 * examined, counts[1] = survivors, counts[2] = survivors under the literal
 * count distance (equal to counts[1] for other variants). */
int orc_filter_stats(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd,
                     const uint8_t *qbytes, const uint64_t *qoffs, uint32_t nq,
                     int variant, uint32_t bits, const uint8_t *map, int metric, uint32_t k,
                     uint64_t counts[3])
{
    if (orc_check_map(map, variant, bits))
        return -1;
    uint32_t *dfp = (uint32_t *)malloc(sizeof(uint32_t) * (nd ? nd : 1));
    if (!dfp)
        return -1;
    orc_fp_many(dbytes, doffs, nd, variant, bits, map, dfp);
    counts[0] = counts[1] = counts[2] = 0;
    for (uint32_t q = 0; q < nq; ++q) {
        uint32_t m = (uint32_t)(qoffs[q + 1] - qoffs[q]);
        uint32_t qfp = orc_fp(qbytes + qoffs[q], m, variant, bits, map);
        for (uint32_t w = 0; w < nd; ++w) {
            uint32_t n = (uint32_t)(doffs[w + 1] - doffs[w]);
            uint32_t gap = m > n ? m - n : n - m;
            int examined = metric == ORC_HAM ? gap == 0 : gap <= k;
            if (!examined)
                continue;
            counts[0]++;
            if (orc_fd(qfp, dfp[w], variant, bits, 0) <= orc_threshold(variant, k))
                counts[1]++;
            if (orc_fd(qfp, dfp[w], variant, bits, 1) <= orc_threshold(variant, k))
                counts[2]++;
        }
    }
    free(dfp);
    return 0;
}

/* Filter statistics under the asymmetric bound: counts[0] = examined
 * (as in orc_filter_stats), counts[1] = pairs with
 * max(excess(q, w), excess(w, q)) <= k. */
int orc_filter_stats_asym(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd,
                          const uint8_t *qbytes, const uint64_t *qoffs, uint32_t nq,
                          int variant, uint32_t bits, const uint8_t *map, int metric, uint32_t k,
                          uint64_t counts[2])
{
    if (orc_check_map(map, variant, bits) || variant == ORC_POS)
        return -1;
    uint32_t *dfp = (uint32_t *)malloc(sizeof(uint32_t) * (nd ? nd : 1));
    if (!dfp)
        return -1;
    orc_fp_many(dbytes, doffs, nd, variant, bits, map, dfp);
    counts[0] = counts[1] = 0;
    for (uint32_t q = 0; q < nq; ++q) {
        uint32_t m = (uint32_t)(qoffs[q + 1] - qoffs[q]);
        uint32_t qfp = orc_fp(qbytes + qoffs[q], m, variant, bits, map);
        for (uint32_t w = 0; w < nd; ++w) {
            uint32_t n = (uint32_t)(doffs[w + 1] - doffs[w]);
            uint32_t gap = m > n ? m - n : n - m;
            int examined = metric == ORC_HAM ? gap == 0 : gap <= k;
            if (!examined)
                continue;
            counts[0]++;
            if (orc_excess(qfp, dfp[w], variant, bits) <= k && orc_excess(dfp[w], qfp, variant, bits) <= k)
                counts[1]++;
        }
    }
    free(dfp);
    return 0;
}

/* F_D of many fingerprint pairs (a[i], b[i]). */
void orc_fd_many(const uint32_t *a, const uint32_t *b, uint64_t n, int variant, uint32_t bits, int literal,
                 uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = orc_fd(a[i], b[i], variant, bits, literal);
}
