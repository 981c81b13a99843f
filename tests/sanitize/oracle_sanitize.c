/*
 * Host-side sanitizer driver for the CPU oracle (test infrastructure).
 *
 * Built together with oracle/oracle.c under AddressSanitizer +
 * UndefinedBehaviorSanitizer (and, separately, ThreadSanitizer for the
 * threaded brute-force matcher) by tests/test_oracle_sanitize.py.  It calls
 * every exported oracle function on seeded synthetic inputs -- empty and
 * 255-byte strings, bytes outside the symbol map, empty dictionaries and
 * query sets, every fingerprint variant at 16 and 32 bits, every symbol set --
 * plus the documented error paths, and checks properties the mathematics
 * fixes, so that a run exercises the code paths the sanitizers watch:
 *   - distances (Section 1): identity, symmetry, |m - n| <= Lev <= max(m, n),
 *     Ham infinite exactly when the lengths differ, Lev <= Ham, the triangle
 *     inequality;
 *   - Eq. 1 soundness (Theorems 1 and 2): a pair within k edits has
 *     F_D <= the threshold for every variant (the literal count XOR excepted);
 *   - the brute-force matcher: thread count and the labelled length-pruned
 *     mode leave the result unchanged, every reported triple re-computes, and
 *     the number of triples equals an exhaustive count over all pairs;
 *   - filter statistics: survivors <= examined, every exact match survives.
 * Exit status 0 when every check holds; a sanitizer report aborts the run.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* The oracle's exported functions (oracle/oracle.c has no header). */
uint32_t orc_ham(const uint8_t *a, uint32_t m, const uint8_t *b, uint32_t n);
uint32_t orc_lev(const uint8_t *a, uint32_t m, const uint8_t *b, uint32_t n);
uint32_t orc_host_threads(void);
int orc_match(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd, const uint8_t *qbytes,
              const uint64_t *qoffs, uint32_t nq, int metric, uint32_t k, uint32_t nthreads, int length_pruned,
              uint32_t **out, uint64_t *n_out);
int orc_pair_dist(const uint8_t *dbytes, const uint64_t *doffs, const uint8_t *qbytes, const uint64_t *qoffs,
                  const uint32_t *pairs, uint64_t npairs, int metric, uint32_t *dist);
void orc_free(void *p);
int orc_num_fields(int variant, uint32_t bits);
void orc_histogram(const uint8_t *bytes, const uint64_t *offs, uint32_t n, uint64_t hist[256]);
int orc_select_symbols(const uint64_t hist[256], int variant, uint32_t bits, int symset, uint8_t map[256]);
uint32_t orc_fp(const uint8_t *s, uint32_t n, int variant, uint32_t bits, const uint8_t *map);
int orc_check_map(const uint8_t *map, int variant, uint32_t bits);
int orc_fp_many(const uint8_t *bytes, const uint64_t *offs, uint32_t n, int variant, uint32_t bits,
                const uint8_t *map, uint32_t *out);
uint32_t orc_fd(uint32_t a, uint32_t b, int variant, uint32_t bits, int literal);
uint32_t orc_excess(uint32_t a, uint32_t b, int variant, uint32_t bits);
void orc_excess_many(const uint32_t *a, const uint32_t *b, uint64_t n, int variant, uint32_t bits, uint32_t *out);
uint32_t orc_threshold(int variant, uint32_t k);
int orc_filter_stats(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd, const uint8_t *qbytes,
                     const uint64_t *qoffs, uint32_t nq, int variant, uint32_t bits, const uint8_t *map, int metric,
                     uint32_t k, uint64_t counts[3]);
int orc_filter_stats_asym(const uint8_t *dbytes, const uint64_t *doffs, uint32_t nd, const uint8_t *qbytes,
                          const uint64_t *qoffs, uint32_t nq, int variant, uint32_t bits, const uint8_t *map,
                          int metric, uint32_t k, uint64_t counts[2]);
void orc_fd_many(const uint32_t *a, const uint32_t *b, uint64_t n, int variant, uint32_t bits, int literal,
                 uint32_t *out);

enum { HAM = 0, LEV = 1 };
enum { OCC = 0, COUNT = 1, POS = 2, OCCH = 3, QGRAM = 4, COMBO = 5, NVARIANTS = 6 };
#define INF 0xFFFFFFFFu
#define NONE 0xFFu

static int failures = 0;
#define CHECK(cond, ...)                                                                                      \
    do {                                                                                                      \
        if (!(cond)) {                                                                                        \
            fprintf(stderr, "check failed (%s:%d): %s: ", __FILE__, __LINE__, #cond);                        \
            fprintf(stderr, __VA_ARGS__);                                                                     \
            fputc('\n', stderr);                                                                              \
            if (++failures > 20)                                                                              \
                exit(1);                                                                                      \
        }                                                                                                     \
    } while (0)

/* splitmix64: the seeded generator of this driver's inputs */
static uint64_t rng_state = 0x1711084750000001ull;
static uint64_t rnd(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint32_t below(uint32_t n) { return n ? (uint32_t)(rnd() % n) : 0; }

/* symbols: mostly a small alphabet (so edits collide and matches exist), a
 * few bytes from the whole range (outside any map, above 127, zero) */
static uint8_t symbol(void)
{
    static const char small[] = "etaoinsrhlzq";
    if (below(16) == 0)
        return (uint8_t)below(256);
    return (uint8_t)small[below(sizeof(small) - 1)];
}

typedef struct {
    uint8_t *bytes;
    uint64_t *offs;
    uint32_t n;
    uint64_t cap;
} strset;

static void set_init(strset *s, uint32_t max_strings)
{
    s->cap = 4096;
    s->bytes = malloc(s->cap);
    s->offs = malloc(sizeof(uint64_t) * (max_strings + 1));
    s->offs[0] = 0;
    s->n = 0;
}
static void set_push(strset *s, const uint8_t *p, uint32_t len)
{
    uint64_t end = s->offs[s->n];
    while (end + len > s->cap) {
        s->cap *= 2;
        s->bytes = realloc(s->bytes, s->cap);
    }
    if (len)
        memcpy(s->bytes + end, p, len);
    s->offs[++s->n] = end + len;
}
static void set_free(strset *s)
{
    free(s->bytes);
    free(s->offs);
}

static uint32_t random_string(uint8_t *out, uint32_t maxlen)
{
    uint32_t len = below(maxlen + 1);
    for (uint32_t i = 0; i < len; ++i)
        out[i] = symbol();
    return len;
}

/* applies e random edits (substitutions only when subst_only) to s in place;
 * returns the new length (at most 255) */
static uint32_t edit(uint8_t *s, uint32_t len, uint32_t e, int subst_only)
{
    for (uint32_t t = 0; t < e; ++t) {
        uint32_t op = subst_only ? 0 : below(3);
        if (op == 1 && len == 255)
            op = 0;
        if ((op == 0 || op == 2) && len == 0)
            op = subst_only ? 3 : 1;
        if (op == 0) {
            s[below(len)] = symbol();
        } else if (op == 1) {
            uint32_t p = below(len + 1);
            memmove(s + p + 1, s + p, len - p);
            s[p] = symbol();
            len++;
        } else if (op == 2) {
            uint32_t p = below(len);
            memmove(s + p, s + p + 1, len - p - 1);
            len--;
        }
    }
    return len;
}

static void check_distances(void)
{
    uint8_t a[256], b[256], c[256];
    for (int it = 0; it < 3000; ++it) {
        uint32_t cap = it % 50 == 0 ? 255 : 24;
        uint32_t m = random_string(a, cap), n = random_string(b, cap), l = random_string(c, cap);
        if (it % 7 == 0) { /* a near copy, so small distances occur */
            memcpy(b, a, m);
            n = edit(b, m, below(3), it % 2);
        }
        uint32_t lab = orc_lev(a, m, b, n), lba = orc_lev(b, n, a, m);
        uint32_t hab = orc_ham(a, m, b, n), hba = orc_ham(b, n, a, m);
        uint32_t gap = m > n ? m - n : n - m, mx = m > n ? m : n;
        CHECK(orc_lev(a, m, a, m) == 0 && orc_ham(a, m, a, m) == 0, "identity at length %u", m);
        CHECK(lab == lba && hab == hba, "symmetry %u/%u %u/%u", lab, lba, hab, hba);
        CHECK(gap <= lab && lab <= mx, "lev %u outside [%u, %u]", lab, gap, mx);
        CHECK((hab == INF) == (m != n), "ham %u for lengths %u, %u", hab, m, n);
        CHECK(hab == INF || lab <= hab, "lev %u > ham %u", lab, hab);
        uint32_t lac = orc_lev(a, m, c, l), lbc = orc_lev(b, n, c, l);
        CHECK(lac <= lab + lbc, "triangle %u > %u + %u", lac, lab, lbc);
    }
}

static void check_maps_and_fingerprints(const strset *d)
{
    uint64_t hist[256];
    orc_histogram(d->bytes, d->offs, d->n, hist);
    uint64_t total = 0;
    for (int c = 0; c < 256; ++c)
        total += hist[c];
    CHECK(total == d->offs[d->n], "histogram total %llu", (unsigned long long)total);
    uint8_t map[256];
    CHECK(orc_select_symbols(hist, OCC, 8, 0, map) == -1, "bits 8 accepted");
    CHECK(orc_select_symbols(hist, OCC, 16, 3, map) == -1, "symbol set 3 accepted");
    CHECK(orc_select_symbols(hist, 6, 16, 0, map) == -1, "variant 6 accepted");
    CHECK(orc_num_fields(POS, 16) == 6 && orc_num_fields(POS, 32) == 12, "position fields");
    uint8_t bad[256];
    memset(bad, NONE, sizeof(bad));
    bad['e'] = 40;
    uint32_t sink[4];
    CHECK(orc_check_map(bad, OCC, 32) == -1 && orc_fp_many(d->bytes, d->offs, 1, OCC, 32, bad, sink) == -1,
          "field 40 accepted at 32 bits");

    uint8_t a[512], b[512];
    for (int variant = 0; variant < NVARIANTS; ++variant) {
        for (uint32_t bits = 16; bits <= 32; bits += 16) {
            for (int symset = 0; symset < 3; ++symset) {
                int nf = orc_select_symbols(hist, variant, bits, symset, map);
                CHECK(nf >= 0 && nf <= orc_num_fields(variant, bits), "variant %d bits %u: %d symbols", variant,
                      bits, nf);
                CHECK(orc_check_map(map, variant, bits) == 0, "selected map rejected");
                uint32_t *fp = malloc(sizeof(uint32_t) * (d->n ? d->n : 1));
                CHECK(orc_fp_many(d->bytes, d->offs, d->n, variant, bits, map, fp) == 0, "fp_many failed");
                for (uint32_t i = 0; i < d->n; i += 17) {
                    uint32_t x = orc_fp(d->bytes + d->offs[i], (uint32_t)(d->offs[i + 1] - d->offs[i]), variant,
                                        bits, map);
                    CHECK(x == fp[i], "fp_many differs at %u", i);
                    CHECK(bits == 32 || x < (1u << 16), "16-bit key 0x%x", x);
                }
                /* Eq. 1 soundness on pairs a few edits apart */
                for (int it = 0; it < 400; ++it) {
                    uint32_t m = random_string(a, it % 40 == 0 ? 255 : 30);
                    uint32_t k = 1 + below(3);
                    int ham = it % 3 == 0;
                    memcpy(b, a, m);
                    uint32_t n = edit(b, m, below(k + 1), ham);
                    uint32_t dist = ham ? orc_ham(a, m, b, n) : orc_lev(a, m, b, n);
                    /* position and occurrence-halved keys are sound for
                     * Hamming only (Theorem 2; the halves split at n / 2) */
                    if (dist > k || (!ham && (variant == POS || variant == OCCH)))
                        continue;
                    uint32_t qa = orc_fp(a, m, variant, bits, map), qb = orc_fp(b, n, variant, bits, map);
                    uint32_t f = orc_fd(qa, qb, variant, bits, 0);
                    CHECK(f <= orc_threshold(variant, k), "variant %d bits %u: dist %u, F_D %u > %u", variant,
                          bits, dist, f, orc_threshold(variant, k));
                    CHECK(f == orc_fd(qb, qa, variant, bits, 0), "F_D asymmetric");
                    if (variant == OCC || variant == OCCH || variant == COUNT)
                        CHECK(orc_excess(qa, qb, variant, bits) <= k && orc_excess(qb, qa, variant, bits) <= k,
                              "variant %d: excess above k = %u", variant, k);
                }
                /* the batch forms equal the single ones */
                uint32_t nn = d->n < 64 ? d->n : 64;
                uint32_t fd1[64], fd2[64], ex[64];
                orc_fd_many(fp, fp + (d->n - nn), nn, variant, bits, 1, fd1);
                orc_excess_many(fp, fp + (d->n - nn), nn, variant, bits, ex);
                for (uint32_t i = 0; i < nn; ++i) {
                    fd2[i] = orc_fd(fp[i], fp[d->n - nn + i], variant, bits, 1);
                    CHECK(fd1[i] == fd2[i], "fd_many differs");
                    if (variant != POS)
                        CHECK(ex[i] == orc_excess(fp[i], fp[d->n - nn + i], variant, bits), "excess_many differs");
                }
                free(fp);
            }
        }
    }
}

static void check_match(const strset *d, const strset *q)
{
    uint32_t threads = orc_host_threads();
    CHECK(threads >= 1, "host threads %u", threads);
    for (int metric = HAM; metric <= LEV; ++metric) {
        for (uint32_t k = 0; k <= 2; ++k) {
            uint32_t *r1 = NULL, *r2 = NULL, *r3 = NULL;
            uint64_t n1 = 0, n2 = 0, n3 = 0;
            CHECK(orc_match(d->bytes, d->offs, d->n, q->bytes, q->offs, q->n, metric, k, 1, 0, &r1, &n1) == 0,
                  "match failed");
            CHECK(orc_match(d->bytes, d->offs, d->n, q->bytes, q->offs, q->n, metric, k, 3, 0, &r2, &n2) == 0,
                  "match (3 threads) failed");
            CHECK(orc_match(d->bytes, d->offs, d->n, q->bytes, q->offs, q->n, metric, k, 0, metric == LEV, &r3,
                            &n3) == 0,
                  "match (host threads, pruned) failed");
            CHECK(n1 == n2 && n1 == n3, "match counts %llu %llu %llu", (unsigned long long)n1,
                  (unsigned long long)n2, (unsigned long long)n3);
            if (n1 == n2 && n1 == n3 && n1) {
                CHECK(memcmp(r1, r2, 12 * n1) == 0 && memcmp(r1, r3, 12 * n1) == 0, "match lists differ");
                for (uint64_t i = 1; i < n1; ++i)
                    CHECK(r1[3 * i - 3] < r1[3 * i] || (r1[3 * i - 3] == r1[3 * i] && r1[3 * i - 2] < r1[3 * i + 1]),
                          "not strictly ascending by (query, word) at %llu", (unsigned long long)i);
            }
            /* queries are words up to two edits away, three in four */
            CHECK(metric != LEV || k != 2 || n1 >= 3 * q->n / 4, "only %llu matches at Lev k = 2",
                  (unsigned long long)n1);
            /* exhaustive count over every pair through orc_pair_dist */
            uint64_t npairs = (uint64_t)d->n * q->n, exact = 0;
            uint32_t *pairs = malloc(sizeof(uint32_t) * 2 * (npairs ? npairs : 1));
            uint32_t *dist = malloc(sizeof(uint32_t) * (npairs ? npairs : 1));
            for (uint32_t i = 0; i < q->n; ++i)
                for (uint32_t w = 0; w < d->n; ++w) {
                    pairs[2 * ((uint64_t)i * d->n + w)] = i;
                    pairs[2 * ((uint64_t)i * d->n + w) + 1] = w;
                }
            CHECK(orc_pair_dist(d->bytes, d->offs, q->bytes, q->offs, pairs, npairs, metric, dist) == 0,
                  "pair_dist failed");
            for (uint64_t p = 0; p < npairs; ++p)
                exact += dist[p] != INF && dist[p] <= k;
            CHECK(exact == n1, "metric %d k %u: %llu exact pairs, %llu listed", metric, k,
                  (unsigned long long)exact, (unsigned long long)n1);
            for (uint64_t i = 0; i < n1 && i < npairs; ++i) {
                uint64_t p = (uint64_t)r1[3 * i] * d->n + r1[3 * i + 1];
                CHECK(dist[p] == r1[3 * i + 2], "listed distance %u, recomputed %u", r1[3 * i + 2], dist[p]);
            }
            /* filter statistics: every exact match survives Eq. 1 */
            uint64_t hist[256];
            uint8_t map[256];
            orc_histogram(d->bytes, d->offs, d->n, hist);
            for (int variant = 0; variant < NVARIANTS; ++variant) {
                orc_select_symbols(hist, variant, 32, 2, map);
                uint64_t c3[3], c2[2];
                CHECK(orc_filter_stats(d->bytes, d->offs, d->n, q->bytes, q->offs, q->n, variant, 32, map, metric,
                                       k, c3) == 0,
                      "filter_stats failed");
                int sound = metric == HAM || (variant != POS && variant != OCCH);
                CHECK(c3[1] <= c3[0] && (!sound || n1 <= c3[1]), "variant %d: %llu examined, %llu survive, %llu match",
                      variant, (unsigned long long)c3[0], (unsigned long long)c3[1], (unsigned long long)n1);
                int rc = orc_filter_stats_asym(d->bytes, d->offs, d->n, q->bytes, q->offs, q->n, variant, 32, map,
                                               metric, k, c2);
                if (variant == POS) {
                    CHECK(rc == -1, "asymmetric bound accepted position keys");
                } else {
                    /* the excess halves are defined for occurrence and count
                     * keys (occurrence-halved: Hamming only) */
                    int bounded = variant == OCC || variant == COUNT || (variant == OCCH && metric == HAM);
                    CHECK(rc == 0 && c2[0] == c3[0] && c2[1] <= c2[0] && (!bounded || n1 <= c2[1]),
                          "variant %d: asymmetric counts", variant);
                }
            }
            free(pairs);
            free(dist);
            orc_free(r1);
            orc_free(r2);
            orc_free(r3);
        }
    }
}

static void check_errors(const strset *d)
{
    strset big;
    set_init(&big, 2);
    uint8_t s[256];
    memset(s, 'e', sizeof(s));
    set_push(&big, s, 255);
    set_push(&big, s, 256); /* one byte over the limit */
    uint32_t *out = (uint32_t *)1;
    uint64_t n = 7;
    CHECK(orc_match(d->bytes, d->offs, d->n, big.bytes, big.offs, 2, LEV, 1, 2, 0, &out, &n) == -1 && !out && !n,
          "256-byte query accepted");
    CHECK(orc_match(big.bytes, big.offs, 2, d->bytes, d->offs, d->n, HAM, 1, 2, 0, &out, &n) == -1,
          "256-byte word accepted");
    CHECK(orc_match(d->bytes, d->offs, d->n, d->bytes, d->offs, d->n, 2, 1, 1, 0, &out, &n) == -1,
          "metric 2 accepted");
    uint32_t pair[2] = {1, 0}, dist = 0;
    CHECK(orc_pair_dist(d->bytes, d->offs, big.bytes, big.offs, pair, 1, LEV, &dist) == -1,
          "256-byte pair accepted");
    pair[0] = 0;
    CHECK(orc_pair_dist(big.bytes, big.offs, big.bytes, big.offs, pair, 1, LEV, &dist) == 0 && dist == 0,
          "255-byte pair distance %u", dist);
    set_free(&big);
}

static void check_empty(const strset *d)
{
    uint64_t zero = 0, c3[3] = {9, 9, 9}, hist[256];
    uint8_t map[256];
    uint32_t *out = NULL;
    uint64_t n = 5;
    orc_histogram(d->bytes, d->offs, d->n, hist);
    orc_select_symbols(hist, OCC, 16, 0, map);
    CHECK(orc_match(d->bytes, &zero, 0, d->bytes, d->offs, d->n, LEV, 2, 2, 0, &out, &n) == 0 && n == 0,
          "empty dictionary");
    orc_free(out);
    CHECK(orc_match(d->bytes, d->offs, d->n, d->bytes, &zero, 0, HAM, 2, 2, 0, &out, &n) == 0 && n == 0,
          "empty query set");
    orc_free(out);
    CHECK(orc_filter_stats(d->bytes, &zero, 0, d->bytes, d->offs, d->n, OCC, 16, map, LEV, 1, c3) == 0 &&
              c3[0] == 0 && c3[1] == 0,
          "empty dictionary statistics");
    uint64_t h0[256];
    orc_histogram(d->bytes, &zero, 0, h0);
    CHECK(orc_select_symbols(h0, OCC, 16, 2, map) == 0, "symbols chosen from an empty histogram");
    CHECK(orc_fp(d->bytes, 0, POS, 32, map) == orc_fp(d->bytes, 0, POS, 32, map), "empty string key");
}

int main(void)
{
    strset d, q;
    set_init(&d, 400);
    set_init(&q, 60);
    uint8_t s[256];
    for (uint32_t i = 0; i < 400; ++i) {
        uint32_t len = i == 0 ? 0 : i == 1 ? 255 : i % 5 == 0 ? 8 : 1 + below(12);
        for (uint32_t t = 0; t < len; ++t)
            s[t] = symbol();
        set_push(&d, s, len);
    }
    for (uint32_t i = 0; i < 60; ++i) { /* queries: near copies of words, some random */
        uint32_t w = below(d.n), len = (uint32_t)(d.offs[w + 1] - d.offs[w]);
        memcpy(s, d.bytes + d.offs[w], len);
        if (i % 4 == 3)
            len = random_string(s, 12);
        else
            len = edit(s, len, below(3), i % 2);
        set_push(&q, s, len);
    }
    check_distances();
    check_maps_and_fingerprints(&d);
    check_match(&d, &q);
    check_errors(&d);
    check_empty(&d);
    set_free(&d);
    set_free(&q);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
