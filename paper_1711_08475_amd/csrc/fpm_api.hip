// fpm_api.hip -- host runtime and C ABI of libfpm (declared in fpm.h).
//
// The runtime owns every device buffer: an index holds the length-sorted,
// padded dictionary with its fingerprints and filter keys; a plan holds the
// buffers of one match pipeline (query staging, work list, match keys and
// output), so repeated runs reuse memory, and the batched schedule replays
// one captured hipGraph.
#include <algorithm>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fpm.h"
#include "fpm_host.hpp"
#include "fpm_internal.hpp"

using namespace fpm;

namespace fpm {

thread_local std::string g_last_error;

fpm_status fail(fpm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

fpm_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FPM_ENOMEM : FPM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

namespace {
struct DeviceMemory {
    std::mutex mu;
    std::unordered_map<void *, size_t> live;
    uint64_t in_use = 0;
    uint64_t limit = 0;  // 0: no limit
};
DeviceMemory &device_memory()
{
    static DeviceMemory *m = new DeviceMemory();  // never destroyed: buffers may be freed at process exit
    return *m;
}
}  // namespace

hipError_t dev_alloc(void **p, size_t bytes)
{
    DeviceMemory &m = device_memory();
    std::lock_guard<std::mutex> g(m.mu);
    *p = nullptr;
    if (m.limit && m.in_use + bytes > m.limit)
        return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    m.live[*p] = bytes;
    m.in_use += bytes;
    return hipSuccess;
}

void dev_free(void *p)
{
    DeviceMemory &m = device_memory();
    std::lock_guard<std::mutex> g(m.mu);
    auto it = m.live.find(p);
    if (it != m.live.end()) {
        m.in_use -= it->second;
        m.live.erase(it);
    }
    (void)hipFree(p);
}

}  // namespace fpm

namespace {

constexpr uint32_t kRing = 256;  // kernel-timing event pairs per plan

uint32_t bits_for(uint64_t n)  // bits to index 0..n-1 (at least 1)
{
    uint32_t b = 1;
    while (b < 64 && (1ull << b) < n)
        ++b;
    return b;
}

int key_kind_for(int variant, uint32_t bits)
{
    if (variant == FPM_QGRAM)
        return kQgram32;
    if (variant == FPM_COMBO)
        return kCombo64;
    if (variant == FPM_COUNT && bits == 32)
        return kPop64;
    if (variant == FPM_POS)
        return bits == 16 ? kPos16 : kPos32;
    return kPop32;
}

// Keys for the asymmetric bound; -1 where it is not defined (position).
int key_kind_asym(int variant, uint32_t bits)
{
    if (variant == FPM_POS || variant == FPM_QGRAM || variant == FPM_COMBO)
        return -1;
    if (variant == FPM_COUNT)
        return bits == 32 ? kAsym64 : kAsym32;
    return bits == 16 ? kTherm32 : kAsym32;
}

size_t key_bytes(int kind) { return key_is_64(kind) ? 8 : 4; }

fpm_status check_csr(const uint8_t *bytes, const uint64_t *offsets, uint32_t n, const char *what)
{
    if (!offsets || (n > 0 && !bytes && offsets[n] > offsets[0]))
        return fail(FPM_EINVAL, "%s: null pointer", what);
    for (uint32_t i = 0; i < n; ++i) {
        if (offsets[i + 1] < offsets[i])
            return fail(FPM_EINVAL, "%s: offsets decrease at %u", what, i);
        if (offsets[i + 1] - offsets[i] > (uint64_t)kMaxLen)
            return fail(FPM_EINVAL, "%s: string %u is longer than %d", what, i, kMaxLen);
    }
    return FPM_OK;
}

// Device copy of a length-sorted, padded string set.
struct StrSet {
    uint32_t n = 0, cap_n = 0;
    uint64_t cap_bytes = 0, str_cap = 0;
    uint32_t *len = nullptr, *perm = nullptr, *soff = nullptr, *str = nullptr, *off = nullptr, *bdw = nullptr;
    uint8_t *slen = nullptr;
    void *key = nullptr;
    uint32_t *fp_orig = nullptr;
    uint32_t *inv = nullptr;
    // popcount order inside the length blocks: the reordered strings,
    // permutation and keys (the view then points at these)
    uint32_t *str2 = nullptr, *perm2 = nullptr;
    void *key2 = nullptr;
    bool pop_ordered = false;

    hipError_t alloc(uint32_t max_n, uint64_t max_bytes, int kind, bool want_fp_orig, bool want_inv,
                     bool want_pop_order)
    {
        cap_n = max_n;
        cap_bytes = max_bytes;
        hipError_t e;
        if ((e = dalloc(&len, max_n)) || (e = dalloc(&perm, max_n)) || (e = dalloc(&soff, max_n)) ||
            (e = dalloc(&slen, max_n)) || (e = dalloc(&off, 257)) || (e = dalloc(&bdw, 257)))
            return e;
        // padded strings: a slot of L bytes holds at most L/4 + 3.75 dwords
        // (L = 17: 8 dwords) and at most 64; each of the 256 length blocks
        // adds at most 3 dwords of alignment
        str_cap = std::min<uint64_t>(max_bytes / 4 + 4ull * max_n, (uint64_t)max_n * 64) + 1024 + 16;
        if ((e = dalloc(&str, str_cap)))
            return e;
        // keys carry one filter chunk of padding (read, never used)
        if ((e = dalloc((uint8_t **)&key, ((size_t)max_n + 64) * key_bytes(kind))))
            return e;
        if ((e = hipMemset(key, 0, ((size_t)max_n + 64) * key_bytes(kind))))
            return e;
        if (want_fp_orig && (e = dalloc(&fp_orig, max_n)))
            return e;
        if (want_inv && (e = dalloc(&inv, max_n)))
            return e;
        if (want_pop_order) {
            const size_t kb = ((size_t)max_n + 64) * key_bytes(kind);
            if ((e = dalloc(&str2, str_cap)) || (e = dalloc(&perm2, max_n)) || (e = dalloc((uint8_t **)&key2, kb)) ||
                (e = hipMemset(str2, 0, str_cap * sizeof(uint32_t))) || (e = hipMemset(key2, 0, kb)))
                return e;
        }
        return hipSuccess;
    }
    void release()
    {
        dfree(len);
        dfree(perm);
        dfree(soff);
        dfree(str);
        dfree(off);
        dfree(bdw);
        dfree(slen);
        dfree(key);
        dfree(fp_orig);
        dfree(inv);
        dfree(str2);
        dfree(perm2);
        dfree(key2);
    }
    StrSetView view() const
    {
        if (pop_ordered)
            return StrSetView{perm2, slen, soff, str2, off, key2};
        return StrSetView{perm, slen, soff, str, off, key};
    }
};

// Length sort, padded layout and fingerprints of n device strings.  With
// pop_order (needs the StrSet's ordering buffers) each length block is then
// ordered by the popcount of the filter key into the second buffers, which
// the set's view returns from then on.
void prep_strings(StrSet &S, const uint8_t *d_bytes, const uint64_t *d_offsets, uint32_t n, uint64_t nbytes_limit,
                  const uint8_t *d_map, int variant, uint32_t bits, int kind, bool fingerprints, bool pop_order,
                  uint32_t *err, uint32_t *scratch, hipStream_t s)
{
    S.n = n;
    launch_lengths(d_offsets, n, S.len, err, s);
    launch_length_sort(S.len, n, S.perm, S.off, S.bdw, scratch, s);
    S.pop_ordered = fingerprints && pop_order;
    if (!fingerprints) {
        launch_layout(d_bytes, d_offsets, nbytes_limit, S.perm, S.len, S.off, S.bdw, n, S.slen, S.soff, S.str,
                      S.str_cap, err, s);
        return;
    }
    launch_layout_fp(d_bytes, d_offsets, nbytes_limit, S.perm, S.len, S.off, S.bdw, n, S.slen, S.soff, S.str,
                     S.str_cap, err, d_map, variant, (int)bits, S.fp_orig, S.key, kind, s);
    if (pop_order)
        launch_pop_order(S.off, S.bdw, S.str, S.perm, S.key, kind, S.str2, S.perm2, S.key2, s);
}

struct DevCounters {
    uint64_t n_out, survivors, cells, examined, pruned;
    uint32_t err, n_pairs, n_items, pad;
    uint32_t counters[kStripes * kStripeStride];  // persistent work counters
};

}  // namespace

struct fpm_index {
    uint32_t n = 0;
    int variant = 0;
    uint32_t bits = 16;
    int kind = kPop32;
    int kind_asym = -1;  // keys of the asymmetric bound (-1: not defined)
    uint8_t map[256];
    uint8_t *d_map = nullptr;
    StrSet words;
    uint32_t h_off[257];
    uint32_t wbits = 1;
    int device = 0;
    uint64_t bytes = 0;     // dictionary bytes
    float build_ms = 0.f;   // device time of the build (symbol statistics .. inverse permutation)
    float layout_ms = 0.f;  // of that: length sort, padded layout and fingerprints
};

struct fpm_plan {
    const fpm_index *ix = nullptr;
    uint32_t max_q = 0;
    uint64_t max_bytes = 0;
    int metric = 0;
    uint32_t k = 1;
    fpm_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int kind = kPop32;
    bool asym = false;   // asymmetric bound: query blocks ordered by popcount too
    bool prune = false;  // the paper's rule over popcount-ordered blocks (kernel kind pop_pruned_kind(kind))
    bool pop = false;    // asym || prune: dictionary and query blocks ordered by key popcount
    bool survivors_only = false;
    int mx_width = 0;         // matrix-core filter over keys of this many bits (0: vector ALUs)
    uint8_t *qexp = nullptr;  // its query rows (mx_width bytes each, 64 padding rows)

    StrSet q;
    // asymmetric bound or popcount pruning: the dictionary with every length
    // block ordered by key popcount (own strings, permutation and keys;
    // lengths, slot offsets and block tables are the index's)
    uint32_t *a_perm = nullptr, *a_str = nullptr;
    void *a_key = nullptr;
    uint32_t *scratch = nullptr;
    PairRec *pairs = nullptr;
    DevCounters *ctr = nullptr;
    uint64_t *keys = nullptr, *tmp = nullptr;
    uint32_t *triples = nullptr;
    uint64_t cap = 0;
    int persistent_blocks = 0;

    // last run
    const uint8_t *last_bytes = nullptr;
    const uint64_t *last_offsets = nullptr;
    uint32_t last_nq = 0;
    bool ran = false;
    uint32_t host_items = 0;
    uint64_t host_examined = 0;

    hipGraphExec_t gall = nullptr, gpre = nullptr, gpost = nullptr;
    bool g_valid = false;
    const uint8_t *g_bytes = nullptr;
    const uint64_t *g_offsets = nullptr;
    uint32_t g_nq = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t kev[2][kRing] = {};
    uint64_t runs = 0;
    std::vector<PairRec> h_pairs;
    uint32_t h_hdr[2] = {0, 0};  // host source of an async copy: lives in the plan

    WorkList worklist() { return WorkList{pairs, &ctr->n_pairs, &ctr->n_items, ctr->counters, &ctr->examined}; }

    void drop_graphs()
    {
        for (hipGraphExec_t *g : {&gall, &gpre, &gpost}) {
            if (*g)
                (void)hipGraphExecDestroy(*g);
            *g = nullptr;
        }
        g_valid = false;
    }

    // (Re)allocates the match buffers for cap_entries matches.  The new
    // buffers are taken before the old ones are released, so on failure the
    // plan keeps its previous buffers and capacity and stays usable.  Called
    // only while nothing runs on the plan's stream.
    fpm_status alloc_output(uint64_t cap_entries)
    {
        uint64_t *k2 = nullptr, *t2 = nullptr;
        uint32_t *tr2 = nullptr;
        hipError_t e;
        if ((e = dalloc(&k2, cap_entries)) || (e = dalloc(&t2, cap_entries)) || (e = dalloc(&tr2, cap_entries * 3))) {
            dfree(k2);
            dfree(t2);
            dfree(tr2);
            return hip_fail(e, "match buffer allocation");
        }
        dfree(keys);
        dfree(tmp);
        dfree(triples);
        keys = k2;
        tmp = t2;
        triples = tr2;
        cap = cap_entries;
        drop_graphs();
        return FPM_OK;
    }
};

// ======================================================================
extern "C" {

const char *fpm_last_error(void) { return g_last_error.c_str(); }

void fpm_free(void *p) { free(p); }

int fpm_num_fields(fpm_variant variant, uint32_t bits)
{
    if (bits != 16 && bits != 32)
        return -1;
    switch (variant) {
    case FPM_OCC:
        return (int)bits;
    case FPM_OCCH:
    case FPM_COUNT:
        return (int)bits / 2;
    case FPM_POS:
        return (int)(bits / 3 + bits % 3);
    case FPM_QGRAM:
        return (int)bits;  // hash buckets; the symbol map is not used
    case FPM_COMBO:
        return (int)bits / 2;  // occurrence fields; the first bits/4 also count
    default:
        return -1;
    }
}

fpm_status fpm_select_symbols(const uint8_t *bytes, const uint64_t *offsets, uint32_t n, fpm_variant variant,
                              uint32_t bits, fpm_symbols symbols, uint8_t map_out[256])
{
    g_last_error.clear();
    const int nf = fpm_num_fields(variant, bits);
    if (nf < 0)
        return fail(FPM_EINVAL, "unknown variant %d or bits %u", (int)variant, bits);
    if (symbols < FPM_COMMON || symbols > FPM_MIXED)
        return fail(FPM_EINVAL, "symbol set must be common, rare or mixed");
    if (!map_out)
        return fail(FPM_EINVAL, "null map_out");
    fpm_status st = check_csr(bytes, offsets, n, "dictionary");
    if (st)
        return st;
    const uint64_t nbytes = offsets[n];
    uint8_t *d_bytes = nullptr, *d_map = nullptr;
    uint64_t *d_off = nullptr;
    unsigned long long *d_hist = nullptr;
    hipStream_t s = nullptr;
    auto cleanup = [&]() {
        dfree(d_bytes);
        dfree(d_map);
        dfree(d_off);
        dfree(d_hist);
        if (s)
            (void)hipStreamDestroy(s);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) || (e = dalloc(&d_bytes, nbytes + 4)) ||
        (e = dalloc(&d_off, (size_t)n + 1)) || (e = dalloc(&d_map, 256)) || (e = dalloc(&d_hist, 256))) {
        cleanup();
        return hip_fail(e, "fpm_select_symbols alloc");
    }
    if (nbytes)
        (void)hipMemcpyAsync(d_bytes, bytes, nbytes, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(d_off, offsets, sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s);
    launch_zero(d_hist, 512, s);
    launch_byte_histogram(d_bytes, d_off, n, d_hist, s);
    launch_select_symbols(d_hist, nf, (int)symbols, d_map, s);
    (void)hipMemcpyAsync(map_out, d_map, 256, hipMemcpyDeviceToHost, s);
    e = hipStreamSynchronize(s);
    cleanup();
    if (e)
        return hip_fail(e, "fpm_select_symbols");
    return FPM_OK;
}

void fpm_index_destroy(fpm_index *ix)
{
    if (!ix)
        return;
    ix->words.release();
    dfree(ix->d_map);
    delete ix;
}

fpm_status fpm_build_fingerprints(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_words,
                                  fpm_variant variant, uint32_t bits, fpm_symbols symbols, const uint8_t *custom_map,
                                  fpm_index **out)
{
    g_last_error.clear();
    if (!out)
        return fail(FPM_EINVAL, "null out");
    *out = nullptr;
    const int nf = fpm_num_fields(variant, bits);
    if (nf < 0)
        return fail(FPM_EINVAL, "unknown variant %d or bits %u (16 or 32)", (int)variant, bits);
    if (symbols < FPM_COMMON || symbols > FPM_CUSTOM)
        return fail(FPM_EINVAL, "unknown symbol set %d", (int)symbols);
    if (symbols == FPM_CUSTOM) {
        if (!custom_map)
            return fail(FPM_EINVAL, "custom symbol set needs a map");
        for (int c = 0; c < 256; ++c)
            if (custom_map[c] != 0xFF && custom_map[c] >= nf)
                return fail(FPM_EINVAL, "custom map: byte %d -> field %d, variant has %d fields", c, custom_map[c], nf);
    }
    if (n_words == 0xFFFFFFFFu)
        return fail(FPM_EINVAL, "too many words");
    fpm_status st = check_csr(bytes, offsets, n_words, "dictionary");
    if (st)
        return st;
    const uint64_t nbytes = offsets[n_words];

    fpm_index *ix = new (std::nothrow) fpm_index();
    if (!ix)
        return fail(FPM_ENOMEM, "host allocation");
    ix->n = n_words;
    ix->variant = variant;
    ix->bits = bits;
    ix->kind = key_kind_for(variant, bits);
    ix->kind_asym = key_kind_asym(variant, bits);
    ix->wbits = bits_for(n_words);
    (void)hipGetDevice(&ix->device);

    uint8_t *d_bytes = nullptr;
    uint64_t *d_off = nullptr;
    unsigned long long *d_hist = nullptr;
    uint32_t *scratch = nullptr, *d_err = nullptr;
    hipStream_t s = nullptr;
    auto cleanup = [&]() {
        dfree(d_bytes);
        dfree(d_off);
        dfree(d_hist);
        dfree(scratch);
        dfree(d_err);
        if (s)
            (void)hipStreamDestroy(s);
    };
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    auto cleanup_events = [&]() {
        for (hipEvent_t &v : ev)
            if (v)
                (void)hipEventDestroy(v);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) || (e = hipEventCreate(&ev[0])) ||
        (e = hipEventCreate(&ev[1])) || (e = hipEventCreate(&ev[2])) || (e = dalloc(&d_bytes, nbytes + 4)) ||
        (e = dalloc(&d_off, (size_t)n_words + 1)) || (e = dalloc(&d_hist, 256)) ||
        (e = dalloc(&scratch, kRadixScratch)) || (e = dalloc(&d_err, 1)) || (e = dalloc(&ix->d_map, 256)) ||
        (e = ix->words.alloc(n_words, nbytes, ix->kind, true, true, false))) {
        cleanup_events();
        cleanup();
        fpm_index_destroy(ix);
        return hip_fail(e, "fpm_build_fingerprints alloc");
    }
    ix->bytes = nbytes;
    if (symbols == FPM_CUSTOM)
        (void)hipMemcpyAsync(ix->d_map, custom_map, 256, hipMemcpyHostToDevice, s);
    if (nbytes)
        (void)hipMemcpyAsync(d_bytes, bytes, nbytes, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(d_off, offsets, sizeof(uint64_t) * ((size_t)n_words + 1), hipMemcpyHostToDevice, s);
    // the device part of the build, timed from here (inputs resident)
    (void)hipEventRecord(ev[0], s);
    launch_zero(d_err, 1, s);
    if (symbols != FPM_CUSTOM) {
        launch_zero(d_hist, 512, s);
        launch_byte_histogram(d_bytes, d_off, n_words, d_hist, s);
        launch_select_symbols(d_hist, nf, (int)symbols, ix->d_map, s);
    }
    (void)hipEventRecord(ev[1], s);
    prep_strings(ix->words, d_bytes, d_off, n_words, nbytes, ix->d_map, variant, bits, ix->kind, true, false, d_err,
                 scratch, s);
    launch_invert(ix->words.perm, n_words, ix->words.inv, s);
    (void)hipEventRecord(ev[2], s);
    uint32_t h_err = 0;
    (void)hipMemcpyAsync(ix->map, ix->d_map, 256, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(ix->h_off, ix->words.off, sizeof(uint32_t) * 257, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&h_err, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    e = hipStreamSynchronize(s);
    if (!e)
        e = hipGetLastError();
    if (!e)
        e = hipEventElapsedTime(&ix->build_ms, ev[0], ev[2]);
    if (!e)
        e = hipEventElapsedTime(&ix->layout_ms, ev[1], ev[2]);
    cleanup_events();
    cleanup();
    if (e) {
        fpm_index_destroy(ix);
        return hip_fail(e, "fpm_build_fingerprints");
    }
    if (h_err) {  // the host checks above leave only a layout overflow
        fpm_index_destroy(ix);
        return fail(FPM_EDEVICE, "fpm_build_fingerprints: padded layout failed (flags %u)", h_err);
    }
    *out = ix;
    return FPM_OK;
}

fpm_status fpm_get_fingerprints(const fpm_index *ix, uint32_t *out)
{
    g_last_error.clear();
    if (!ix || (!out && ix->n))
        return fail(FPM_EINVAL, "null pointer");
    if (ix->n)
        HIPCHK(hipMemcpy(out, ix->words.fp_orig, sizeof(uint32_t) * ix->n, hipMemcpyDeviceToHost));
    return FPM_OK;
}

fpm_status fpm_get_map(const fpm_index *ix, uint8_t map_out[256])
{
    g_last_error.clear();
    if (!ix || !map_out)
        return fail(FPM_EINVAL, "null pointer");
    memcpy(map_out, ix->map, 256);
    return FPM_OK;
}

fpm_status fpm_index_build_ms(const fpm_index *ix, float *total_ms, float *layout_ms)
{
    g_last_error.clear();
    if (!ix)
        return fail(FPM_EINVAL, "null index");
    if (total_ms)
        *total_ms = ix->build_ms;
    if (layout_ms)
        *layout_ms = ix->layout_ms;
    return FPM_OK;
}

fpm_status fpm_set_device_memory_limit(uint64_t max_bytes)
{
    g_last_error.clear();
    DeviceMemory &m = device_memory();
    std::lock_guard<std::mutex> g(m.mu);
    m.limit = max_bytes;
    return FPM_OK;
}

fpm_status fpm_device_memory_in_use(uint64_t *bytes)
{
    g_last_error.clear();
    if (!bytes)
        return fail(FPM_EINVAL, "null pointer");
    DeviceMemory &m = device_memory();
    std::lock_guard<std::mutex> g(m.mu);
    *bytes = m.in_use;
    return FPM_OK;
}

fpm_status fpm_index_info(const fpm_index *ix, uint32_t *n_words, uint32_t *variant, uint32_t *bits)
{
    g_last_error.clear();
    if (!ix)
        return fail(FPM_EINVAL, "null index");
    if (n_words)
        *n_words = ix->n;
    if (variant)
        *variant = (uint32_t)ix->variant;
    if (bits)
        *bits = ix->bits;
    return FPM_OK;
}

// ---------------------------------------------------------------- plans

static void plan_free(fpm_plan *p)
{
    if (!p)
        return;
    p->drop_graphs();
    for (int i = 0; i < 2; ++i)
        for (uint32_t j = 0; j < kRing; ++j)
            if (p->kev[i][j])
                (void)hipEventDestroy(p->kev[i][j]);
    p->q.release();
    dfree(p->a_perm);
    dfree(p->a_str);
    dfree(p->a_key);
    dfree(p->scratch);
    dfree(p->pairs);
    dfree(p->ctr);
    dfree(p->keys);
    dfree(p->tmp);
    dfree(p->triples);
    dfree(p->qexp);
    if (p->ev0)
        (void)hipEventDestroy(p->ev0);
    if (p->ev1)
        (void)hipEventDestroy(p->ev1);
    if (p->own_stream && p->stream)
        (void)hipStreamDestroy(p->stream);
    delete p;
}

void fpm_plan_destroy(fpm_plan *plan) { plan_free(plan); }

static fpm_status check_metric(const fpm_index *ix, fpm_metric metric, uint32_t k)
{
    if (metric != FPM_HAM && metric != FPM_LEV)
        return fail(FPM_EINVAL, "unknown metric %d", (int)metric);
    if (k < 1 || k > (uint32_t)kMaxK)
        return fail(FPM_EUNSUPPORTED, "k = %u: the GPU matcher supports k = 1 .. %d", k, kMaxK);
    if (metric == FPM_LEV && (ix->variant == FPM_POS || ix->variant == FPM_OCCH))
        return fail(FPM_EUNSUPPORTED, "position and occurrence-halved fingerprints are sound for Hamming only");
    return FPM_OK;
}

static fpm_status resolve_options(const fpm_options *in, fpm_options *o)
{
    memset(o, 0, sizeof(*o));
    if (in)
        *o = *in;
    if (o->schedule > FPM_SCHED_BRUTE)
        return fail(FPM_EINVAL, "unknown schedule %u", o->schedule);
    if (!o->queries_per_item)
        o->queries_per_item = 64;
    if (!o->slab)
        o->slab = 4096;
    if (!o->use_graph)
        o->use_graph = 1;
    if (!o->waves_per_cu)
        o->waves_per_cu = 32;
    if (!o->match_capacity)
        o->match_capacity = 1u << 20;
    if (o->queries_per_item % 16 || o->queries_per_item > 1024)
        return fail(FPM_EINVAL, "queries_per_item must be a multiple of 16 up to 1024");
    if (o->slab % 64 || o->slab < 64 || o->slab > (1u << 22))
        return fail(FPM_EINVAL, "slab must be a multiple of 64 in 64..4M");
    if (o->bucket_order > 1)
        return fail(FPM_EINVAL, "bucket_order must be 0 or 1");
    if (o->waves_per_cu > 64)
        return fail(FPM_EINVAL, "waves_per_cu must be <= 64");
    if (o->time_kernel > 1)
        return fail(FPM_EINVAL, "time_kernel must be 0 or 1");
    if (!o->tail_split)
        o->tail_split = 100;
    if (o->tail_split > 100)
        return fail(FPM_EINVAL, "tail_split must be in 1..100 (0 = default)");
    if (o->bound > FPM_BOUND_ASYM)
        return fail(FPM_EINVAL, "unknown bound %u", o->bound);
    if (o->filter_unit > FPM_UNIT_MATRIX)
        return fail(FPM_EINVAL, "unknown filter unit %u", o->filter_unit);
    if (o->pop_prune > FPM_PRUNE_ON)
        return fail(FPM_EINVAL, "unknown pop_prune %u", o->pop_prune);
    return FPM_OK;
}

// The dictionary of a plan over popcount-ordered blocks (asymmetric bound or
// popcount pruning): the index's length blocks, each ordered by key popcount
// (stable), with keys of the plan's family.  Runs once at plan creation and
// waits for it.
static fpm_status build_pop_dictionary(fpm_plan *p)
{
    const fpm_index *ix = p->ix;
    const StrSet &W = ix->words;
    const uint32_t n = ix->n;
    hipStream_t s = p->stream;
    const size_t kb = ((size_t)n + 64) * key_bytes(p->kind);  // same width as the index's keys
    hipError_t e;
    if ((e = dalloc(&p->a_perm, std::max<uint32_t>(n, 1))) || (e = dalloc(&p->a_str, W.str_cap)) ||
        (e = dalloc((uint8_t **)&p->a_key, kb)) ||
        (e = hipMemsetAsync(p->a_str, 0, W.str_cap * sizeof(uint32_t), s)) || (e = hipMemsetAsync(p->a_key, 0, kb, s)))
        return hip_fail(e, "popcount-ordered dictionary alloc");
    launch_pop_order(W.off, W.bdw, W.str, W.perm, W.key, ix->kind, p->a_str, p->a_perm, p->a_key, s);
    if (p->kind == kTherm32)  // the moved keys are the plain ones: extend them
        launch_fingerprints(p->a_str, W.soff, W.slen, p->a_perm, n, ix->d_map, ix->variant, (int)ix->bits, nullptr,
                            nullptr, p->a_key, p->kind, s);
    e = hipStreamSynchronize(s);
    if (!e)
        e = hipGetLastError();
    if (e)
        return hip_fail(e, "popcount-ordered dictionary");
    return FPM_OK;
}

static fpm_status plan_create(const fpm_index *ix, uint32_t max_queries, uint64_t max_query_bytes, fpm_metric metric,
                              uint32_t k, const fpm_options *opt, void *hip_stream, bool survivors_only,
                              fpm_plan **out)
{
    if (!out)
        return fail(FPM_EINVAL, "null out");
    *out = nullptr;
    if (!ix)
        return fail(FPM_EINVAL, "null index");
    fpm_status st = check_metric(ix, metric, k);
    if (st)
        return st;
    if (max_queries >= (1u << 30))
        return fail(FPM_EINVAL, "max_queries must be below 2^30");
    if (bits_for(std::max<uint32_t>(max_queries, 1)) + ix->wbits + 2 > 64)
        return fail(FPM_EINVAL, "query and word index bits exceed the 64-bit match key");
    fpm_plan *p = new (std::nothrow) fpm_plan();
    if (!p)
        return fail(FPM_ENOMEM, "host allocation");
    st = resolve_options(opt, &p->opt);
    if (st) {
        delete p;
        return st;
    }
    p->ix = ix;
    p->max_q = max_queries;
    p->max_bytes = max_query_bytes;
    p->metric = metric;
    p->k = k;
    p->survivors_only = survivors_only;
    p->asym = p->opt.bound == FPM_BOUND_ASYM && p->opt.schedule != FPM_SCHED_BRUTE;
    if (p->asym && ix->kind_asym < 0) {
        delete p;
        return fail(FPM_EUNSUPPORTED, "the asymmetric bound is offered for occurrence, occurrence-halved and count "
                                      "fingerprints only");
    }
    p->kind = p->opt.schedule == FPM_SCHED_BRUTE ? kAll : p->asym ? ix->kind_asym : ix->kind;
    // the matrix-core filter: the paper's rule on keys of up to 32 bits whose
    // F_D is the popcount of their XOR (16-bit count keys are 24-bit
    // thermometer codes: 32-bit tiles)
    const bool mx_ok = !p->asym && (p->kind == kPop32 || p->kind == kQgram32);
    if (p->opt.filter_unit == FPM_UNIT_MATRIX && !mx_ok) {
        delete p;
        return fail(FPM_EUNSUPPORTED, "the matrix-core filter takes the paper's rule on occurrence, "
                                      "occurrence-halved, 16-bit count and bigram fingerprints");
    }
    // auto: the vector ALUs (the method is integer bit arithmetic); the
    // matrix cores only when asked for
    const int key_width = ix->bits == 16 && ix->variant != FPM_COUNT ? 16 : 32;
    p->mx_width = mx_ok && p->opt.filter_unit == FPM_UNIT_MATRIX ? key_width : 0;
    // the matrix-core kernels hold 7 blocks per compute unit (their register
    // budget), the vector-ALU kernels 8
    if (p->mx_width && !(opt && opt->waves_per_cu))
        p->opt.waves_per_cu = 28;
    // popcount pruning (on request): the batched schedule, for keys whose
    // F_D is the popcount of their XOR
    const bool prune_ok = !p->asym && p->opt.schedule == FPM_SCHED_BATCHED && pop_pruned_kind(p->kind) >= 0;
    if (p->opt.pop_prune == FPM_PRUNE_ON && !prune_ok) {
        delete p;
        return fail(FPM_EUNSUPPORTED, "popcount pruning takes the batched schedule with occurrence, "
                                      "occurrence-halved, count or bigram fingerprints and the paper's rule");
    }
    p->prune = p->opt.pop_prune == FPM_PRUNE_ON;
    p->pop = p->asym || p->prune;
    hipError_t e = hipSuccess;
    if (hip_stream) {
        p->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        p->own_stream = true;
    }
    const int qkind = p->kind == kAll ? kPop32 : p->kind;
    if (e || (e = p->q.alloc(max_queries, max_query_bytes, qkind, false, false, p->pop)) ||
        (e = dalloc(&p->scratch, kRadixScratch)) || (e = dalloc(&p->pairs, kMaxPairs)) ||
        (e = dalloc(&p->ctr, 1)) || (e = hipEventCreate(&p->ev0)) || (e = hipEventCreate(&p->ev1))) {
        plan_free(p);
        return hip_fail(e, "fpm_plan_create alloc");
    }
    if (p->mx_width) {
        const size_t qb = ((size_t)max_queries + 64) * kMxRowBytes;
        if ((e = dalloc(&p->qexp, qb)) || (e = hipMemset(p->qexp, 0, qb))) {
            plan_free(p);
            return hip_fail(e, "fpm_plan_create alloc");
        }
    }
    p->q.pop_ordered = p->pop;
    st = p->alloc_output(p->opt.match_capacity);
    if (!st && p->pop)
        st = build_pop_dictionary(p);
    if (st) {
        plan_free(p);
        return st;
    }
    if (p->opt.time_kernel == 1) {
        for (int i = 0; i < 2; ++i)
            for (uint32_t j = 0; j < kRing; ++j)
                if ((e = hipEventCreate(&p->kev[i][j]))) {
                    plan_free(p);
                    return hip_fail(e, "kernel timing events");
                }
    }
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ix->device) == hipSuccess)
        cus = prop.multiProcessorCount;
    p->persistent_blocks = std::max(1, cus * (int)p->opt.waves_per_cu / 4);
    p->h_pairs.resize(kMaxPairs);
    *out = p;
    return FPM_OK;
}

fpm_status fpm_plan_create(const fpm_index *ix, uint32_t max_queries, uint64_t max_query_bytes, fpm_metric metric,
                           uint32_t k, const fpm_options *opt, void *hip_stream, fpm_plan **out)
{
    g_last_error.clear();
    return plan_create(ix, max_queries, max_query_bytes, metric, k, opt, hip_stream, false, out);
}

// The device work of one match in three parts: prep (query staging,
// fingerprints, work list), the match kernel, post (sort, unpack).  With
// `plain` the host reads the query bucket table during prep (one
// synchronisation).
static fpm_status enqueue_prep(fpm_plan *p, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t nq,
                               bool plain)
{
    const fpm_index *ix = p->ix;
    hipStream_t s = p->stream;
    launch_zero(p->ctr, sizeof(DevCounters) / 4, s);
    const bool fps = p->kind != kAll;
    prep_strings(p->q, d_qbytes, d_qoffsets, nq, p->max_bytes, ix->d_map, ix->variant, ix->bits,
                 fps ? p->kind : kPop32, fps, p->pop, &p->ctr->err, p->scratch, s);
    if (p->mx_width)
        // the rows follow the order the kernel reads the queries in (the
        // popcount order when the blocks are ordered)
        launch_expand_keys((const uint32_t *)p->q.view().key, nq, p->mx_width, p->qexp, s);
    if (plain) {
        uint32_t h_qoff[257];
        HIPCHK(hipMemcpyAsync(h_qoff, p->q.off, sizeof(h_qoff), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        uint32_t np = 0;
        p->host_items = host_worklist(h_qoff, ix->h_off, p->metric, p->k, p->opt.queries_per_item, p->opt.slab,
                                      p->opt.bucket_order, p->h_pairs.data(), &np, &p->host_examined);
        p->h_hdr[0] = np;
        p->h_hdr[1] = p->host_items;
        if (np)
            HIPCHK(hipMemcpyAsync(p->pairs, p->h_pairs.data(), sizeof(PairRec) * np, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(&p->ctr->n_pairs, p->h_hdr, sizeof(p->h_hdr), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(&p->ctr->examined, &p->host_examined, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    } else {
        launch_worklist(p->q.off, ix->words.off, p->metric, p->k, p->opt.queries_per_item, p->opt.slab,
                        p->opt.bucket_order, p->opt.tail_split >= 100 ? 0u : p->opt.tail_split, p->worklist(), s);
    }
    return FPM_OK;
}

static fpm_status enqueue_kernel(fpm_plan *p, bool plain)
{
    const fpm_index *ix = p->ix;
    MatchArgs a;
    a.q = p->q.view();
    a.d = ix->words.view();
    if (p->pop) {
        a.d.perm = p->a_perm;
        a.d.str = p->a_str;
        a.d.key = p->a_key;
    }
    a.wl = p->worklist();
    a.ctr = MatchCounters{&p->ctr->n_out, &p->ctr->survivors, &p->ctr->cells, &p->ctr->pruned};
    a.out_keys = p->keys;
    a.out_cap = p->cap;
    a.wbits = ix->wbits;
    a.survivors_only = p->survivors_only ? 1u : 0u;
    a.qexp = p->qexp;
    hipError_t e = launch_match(a, p->prune ? pop_pruned_kind(p->kind) : p->kind, p->mx_width, p->metric, p->k,
                                !plain, (uint32_t)p->persistent_blocks, p->host_items, p->stream);
    if (e)
        return hip_fail(e, "match kernel launch");
    return FPM_OK;
}

static void enqueue_post(fpm_plan *p, uint32_t nq)
{
    const fpm_index *ix = p->ix;
    const uint32_t qbits = bits_for(std::max<uint32_t>(nq, 1));
    launch_sort_unpack(p->keys, p->tmp, &p->ctr->n_out, p->cap, 2, 2 + ix->wbits + qbits, ix->wbits, p->triples,
                       p->survivors_only ? 1 : 0, p->scratch, p->stream);
}

static fpm_status capture(fpm_plan *p, hipGraphExec_t *out, int part, const uint8_t *b, const uint64_t *o,
                          uint32_t nq)
{
    hipStream_t s = p->stream;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    fpm_status st = FPM_OK;
    if (part & 1)
        st = enqueue_prep(p, b, o, nq, false);
    if (!st && (part & 2))
        st = enqueue_kernel(p, false);
    if (!st && (part & 4))
        enqueue_post(p, nq);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e)
        return hip_fail(e, "graph capture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e)
        return hip_fail(e, "graph instantiate");
    return FPM_OK;
}

static fpm_status plan_launch(fpm_plan *p, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t nq)
{
    hipStream_t s = p->stream;
    const bool plain = p->opt.schedule != FPM_SCHED_BATCHED;
    const bool graph = !plain && p->opt.use_graph == 1;
    const bool timed = p->opt.time_kernel == 1;
    const uint32_t slot = (uint32_t)(p->runs % kRing);
    HIPCHK(hipEventRecord(p->ev0, s));
    if (graph) {
        if (!p->g_valid || p->g_bytes != d_qbytes || p->g_offsets != d_qoffsets || p->g_nq != nq) {
            p->drop_graphs();
            fpm_status st = timed ? capture(p, &p->gpre, 1, d_qbytes, d_qoffsets, nq)
                                  : capture(p, &p->gall, 7, d_qbytes, d_qoffsets, nq);
            if (!st && timed)
                st = capture(p, &p->gpost, 4, d_qbytes, d_qoffsets, nq);
            if (st)
                return st;
            p->g_valid = true;
            p->g_bytes = d_qbytes;
            p->g_offsets = d_qoffsets;
            p->g_nq = nq;
        }
        if (timed) {
            HIPCHK(hipGraphLaunch(p->gpre, s));
            HIPCHK(hipEventRecord(p->kev[0][slot], s));
            fpm_status st = enqueue_kernel(p, false);
            if (st)
                return st;
            HIPCHK(hipEventRecord(p->kev[1][slot], s));
            HIPCHK(hipGraphLaunch(p->gpost, s));
        } else {
            HIPCHK(hipGraphLaunch(p->gall, s));
        }
    } else {
        fpm_status st = enqueue_prep(p, d_qbytes, d_qoffsets, nq, plain);
        if (st)
            return st;
        if (timed)
            HIPCHK(hipEventRecord(p->kev[0][slot], s));
        st = enqueue_kernel(p, plain);
        if (st)
            return st;
        if (timed)
            HIPCHK(hipEventRecord(p->kev[1][slot], s));
        enqueue_post(p, nq);
    }
    HIPCHK(hipEventRecord(p->ev1, s));
    if (timed)
        p->runs++;
    return FPM_OK;
}

fpm_status fpm_plan_kernel_ms(fpm_plan *p, float *ms_out, uint32_t max, uint32_t *n)
{
    g_last_error.clear();
    if (!p || (max && !ms_out))
        return fail(FPM_EINVAL, "null pointer");
    if (p->opt.time_kernel != 1)
        return fail(FPM_EINVAL, "plan was created without time_kernel");
    HIPCHK(hipStreamSynchronize(p->stream));
    const uint64_t avail = std::min<uint64_t>(p->runs, kRing);
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(avail, max);
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t slot = (uint32_t)((p->runs - cnt + i) % kRing);
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p->kev[0][slot], p->kev[1][slot]));
        ms_out[i] = ms;
    }
    if (n)
        *n = cnt;
    return FPM_OK;
}

fpm_status fpm_plan_run(fpm_plan *p, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t n_queries)
{
    g_last_error.clear();
    if (!p)
        return fail(FPM_EINVAL, "null plan");
    if (n_queries > p->max_q)
        return fail(FPM_EINVAL, "%u queries exceed the plan's %u", n_queries, p->max_q);
    if (n_queries && (!d_qoffsets || (!d_qbytes && p->max_bytes)))
        return fail(FPM_EINVAL, "null query pointer");
    p->last_bytes = d_qbytes;
    p->last_offsets = d_qoffsets;
    p->last_nq = n_queries;
    p->ran = true;
    if (n_queries == 0)
        return FPM_OK;
    return plan_launch(p, d_qbytes, d_qoffsets, n_queries);
}

fpm_status fpm_plan_result(fpm_plan *p, const fpm_hit **d_matches, uint64_t *n_out, fpm_stats *stats)
{
    g_last_error.clear();
    if (!p || !p->ran)
        return fail(FPM_EINVAL, "plan has not run");
    fpm_stats st;
    memset(&st, 0, sizeof(st));
    st.pairs_logical = (uint64_t)p->last_nq * p->ix->n;
    if (p->last_nq == 0) {
        if (d_matches)
            *d_matches = (const fpm_hit *)p->triples;
        if (n_out)
            *n_out = 0;
        if (stats)
            *stats = st;
        return FPM_OK;
    }
    DevCounters c;
    for (int attempt = 0; attempt < 3; ++attempt) {
        HIPCHK(hipStreamSynchronize(p->stream));
        HIPCHK(hipMemcpy(&c, p->ctr, offsetof(DevCounters, counters), hipMemcpyDeviceToHost));
        if (c.err)
            return fail(FPM_EINVAL, "query batch: %s",
                        (c.err & 2) ? "offsets decrease"
                                    : (c.err & 1) ? "a string is longer than 255" : "more bytes than max_query_bytes");
        if (c.n_out <= p->cap)
            break;
        // the match buffer overflowed: grow it and run again
        fpm_status s2 = p->alloc_output(c.n_out + c.n_out / 4 + 1024);
        if (s2)
            return s2;
        s2 = plan_launch(p, p->last_bytes, p->last_offsets, p->last_nq);
        if (s2)
            return s2;
    }
    if (c.n_out > p->cap)
        return fail(FPM_EDEVICE, "match buffer overflow persists");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev0, p->ev1);
    st.pairs_examined = c.examined;
    st.survivors = c.survivors;
    st.matches = c.n_out;
    st.verify_cells = c.cells;
    st.pairs_filtered = p->kind == kAll ? 0 : c.examined - std::min(c.pruned, c.examined);
    st.ms = ms;
    st.work_items = c.n_items;
    st.filter_unit = p->kind == kAll ? FPM_UNIT_AUTO : p->mx_width ? FPM_UNIT_MATRIX : FPM_UNIT_VALU;
    if (d_matches)
        *d_matches = (const fpm_hit *)p->triples;
    if (n_out)
        *n_out = c.n_out;
    if (stats)
        *stats = st;
    return FPM_OK;
}

fpm_status fpm_plan_copy_matches(fpm_plan *p, fpm_hit *dst, uint64_t max, uint64_t *n_copied)
{
    g_last_error.clear();
    const fpm_hit *dm = nullptr;
    uint64_t n = 0;
    fpm_status st = fpm_plan_result(p, &dm, &n, nullptr);
    if (st)
        return st;
    n = std::min(n, max);
    if (n) {
        if (!dst)
            return fail(FPM_EINVAL, "null destination");
        HIPCHK(hipMemcpy(dst, dm, sizeof(fpm_hit) * n, hipMemcpyDefault));
    }
    if (n_copied)
        *n_copied = n;
    return FPM_OK;
}

// Host-buffer convenience path: one temporary plan per call.
static fpm_status match_host(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t nq,
                             fpm_metric metric, uint32_t k, const fpm_options *opt, bool survivors_only,
                             uint32_t **out, uint64_t *n_out, fpm_stats *stats)
{
    if (!ix || !out || !n_out)
        return fail(FPM_EINVAL, "null pointer");
    *out = nullptr;
    *n_out = 0;
    fpm_status st = check_metric(ix, metric, k);
    if (st)
        return st;
    st = check_csr(qbytes, qoffsets, nq, "queries");
    if (st)
        return st;
    const uint64_t nbytes = nq ? qoffsets[nq] : 0;
    fpm_plan *p = nullptr;
    st = plan_create(ix, std::max<uint32_t>(nq, 1), nbytes + 4, metric, k, opt, nullptr, survivors_only, &p);
    if (st)
        return st;
    uint8_t *d_b = nullptr;
    uint64_t *d_o = nullptr;
    hipError_t e;
    if ((e = dalloc(&d_b, nbytes + 4)) || (e = dalloc(&d_o, (size_t)nq + 1))) {
        dfree(d_b);
        plan_free(p);
        return hip_fail(e, "query upload alloc");
    }
    if (nbytes)
        (void)hipMemcpyAsync(d_b, qbytes, nbytes, hipMemcpyHostToDevice, p->stream);
    if (nq)
        (void)hipMemcpyAsync(d_o, qoffsets, sizeof(uint64_t) * ((size_t)nq + 1), hipMemcpyHostToDevice, p->stream);
    st = fpm_plan_run(p, d_b, d_o, nq);
    const fpm_hit *dm = nullptr;
    uint64_t n = 0;
    if (!st)
        st = fpm_plan_result(p, &dm, &n, stats);
    if (!st && n) {
        const size_t width = survivors_only ? 2 : 3;
        uint32_t *h = (uint32_t *)malloc(sizeof(uint32_t) * width * n);
        if (!h) {
            st = fail(FPM_ENOMEM, "host result allocation");
        } else if ((e = hipMemcpy(h, dm, sizeof(uint32_t) * width * n, hipMemcpyDeviceToHost))) {
            free(h);
            st = hip_fail(e, "result copy");
        } else {
            *out = h;
            *n_out = n;
        }
    }
    dfree(d_b);
    dfree(d_o);
    plan_free(p);
    return st;
}

fpm_status fpm_match(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                     fpm_metric metric, uint32_t k, const fpm_options *opt, fpm_hit **out, uint64_t *n_out,
                     fpm_stats *stats)
{
    g_last_error.clear();
    return match_host(ix, qbytes, qoffsets, n_queries, metric, k, opt, false, (uint32_t **)out, n_out, stats);
}

fpm_status fpm_filter_pairs(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets,
                            uint32_t n_queries, fpm_metric metric, uint32_t k, uint32_t **pairs, uint64_t *n_pairs)
{
    g_last_error.clear();
    fpm_options o;
    memset(&o, 0, sizeof(o));
    o.schedule = FPM_SCHED_PLAIN;
    return match_host(ix, qbytes, qoffsets, n_queries, metric, k, &o, true, pairs, n_pairs, nullptr);
}

// ---------------------------------------------------- allocation-free match
//
// fpm_match_noalloc keeps every intermediate buffer of one match (the query
// batch's sorted padded strings and keys, the radix scratch, the work list,
// the counters, the match keys and, for the matrix-core filter, the
// expanded query rows) in one file-scope device array, `scratch`, carved at
// fixed offsets for the limits below.  Host code never passes the array's
// name to a kernel: its device address comes from hipGetSymbolAddress, once
// per device, and only that address is used.

}  // extern "C"

namespace {

constexpr uint32_t kNaMaxQueries = FPM_NOALLOC_MAX_QUERIES;
constexpr uint64_t kNaMaxQueryBytes = FPM_NOALLOC_MAX_QUERY_BYTES;
constexpr uint64_t kNaMaxMatches = FPM_NOALLOC_MAX_MATCHES;
constexpr int kNaMaxDevices = 64;

constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the carved buffers (sizes as StrSet::alloc and
// plan_create would allocate them for the limits).
struct NaLayout {
    size_t len, perm, soff, slen, off, bdw, str, key, radix, pairs, ctr, keys, tmp, qexp, total;
    uint64_t str_cap;  // dwords
};

constexpr NaLayout na_layout()
{
    NaLayout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o += na_align(bytes);
        return at;
    };
    L.str_cap = std::min<uint64_t>(kNaMaxQueryBytes / 4 + 4ull * kNaMaxQueries, (uint64_t)kNaMaxQueries * 64) + 1024 +
                16;
    L.len = take(4ull * kNaMaxQueries);
    L.perm = take(4ull * kNaMaxQueries);
    L.soff = take(4ull * kNaMaxQueries);
    L.slen = take(kNaMaxQueries);
    L.off = take(4 * 257);
    L.bdw = take(4 * 257);
    L.str = take(4 * L.str_cap);
    L.key = take(8ull * (kNaMaxQueries + 64));
    L.radix = take(4 * kRadixScratch);
    L.pairs = take(sizeof(PairRec) * kMaxPairs);
    L.ctr = take(sizeof(DevCounters));
    L.keys = take(8 * kNaMaxMatches);
    L.tmp = take(8 * kNaMaxMatches);
    L.qexp = take((size_t)(kNaMaxQueries + 64) * kMxRowBytes);
    L.total = o;
    return L;
}

constexpr NaLayout kNa = na_layout();

// The library's allocation-free working memory (each device holds its own
// copy from the time the library is loaded until the process ends).
static __device__ __align__(256) uint8_t scratch[kNa.total];

struct NaDevice {
    std::mutex mu;             // calls on one device run one at a time
    uint8_t *base = nullptr;   // device address of `scratch` on this device
    int cus = 0;
};
NaDevice g_na[kNaMaxDevices];

}  // namespace

extern "C" {

fpm_status fpm_match_noalloc(const fpm_index *ix, const uint8_t *d_qbytes, const uint64_t *d_qoffsets,
                             uint32_t n_queries, uint64_t query_bytes, fpm_metric metric, uint32_t k,
                             const fpm_options *opt, void *hip_stream, fpm_hit *d_out, uint64_t out_cap,
                             uint64_t *n_out, fpm_stats *stats)
{
    g_last_error.clear();
    if (!ix || !n_out)
        return fail(FPM_EINVAL, "null pointer");
    *n_out = 0;
    fpm_status st = check_metric(ix, metric, k);
    if (st)
        return st;
    if (n_queries > kNaMaxQueries)
        return fail(FPM_EINVAL, "%u queries exceed the allocation-free limit of %u", n_queries, kNaMaxQueries);
    if (query_bytes > kNaMaxQueryBytes)
        return fail(FPM_EINVAL, "%llu query bytes exceed the allocation-free limit of %llu",
                    (unsigned long long)query_bytes, (unsigned long long)kNaMaxQueryBytes);
    if (n_queries && (!d_qoffsets || (!d_qbytes && query_bytes)))
        return fail(FPM_EINVAL, "null query pointer");
    if (out_cap && !d_out)
        return fail(FPM_EINVAL, "null output pointer");
    fpm_options o;
    st = resolve_options(opt, &o);
    if (st)
        return st;
    if (o.bound == FPM_BOUND_ASYM && o.schedule != FPM_SCHED_BRUTE)
        return fail(FPM_EUNSUPPORTED, "the allocation-free match takes the paper's rule only");
    if (o.pop_prune == FPM_PRUNE_ON)
        return fail(FPM_EUNSUPPORTED, "the allocation-free match has no popcount-ordered dictionary");
    const bool mx_ok = ix->kind == kPop32 || ix->kind == kQgram32;
    if (o.filter_unit == FPM_UNIT_MATRIX && o.schedule != FPM_SCHED_BRUTE && !mx_ok)
        return fail(FPM_EUNSUPPORTED, "the matrix-core filter takes the paper's rule on occurrence, "
                                      "occurrence-halved, 16-bit count and bigram fingerprints");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != ix->device)
        return fail(FPM_EINVAL, "the index lives on device %d, device %d is current", ix->device, dev);
    if (dev < 0 || dev >= kNaMaxDevices)
        return fail(FPM_EUNSUPPORTED, "device %d: the allocation-free match supports devices 0..%d", dev,
                    kNaMaxDevices - 1);
    NaDevice &nd = g_na[dev];
    std::lock_guard<std::mutex> lock(nd.mu);
    if (!nd.base) {  // first call on this device: the array's device address
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "allocation-free scratch address");
        hipDeviceProp_t prop;
        nd.cus = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 256;
        nd.base = (uint8_t *)ptr;
    }
    fpm_stats sres;
    memset(&sres, 0, sizeof(sres));
    sres.pairs_logical = (uint64_t)n_queries * ix->n;
    if (n_queries == 0) {
        if (stats)
            *stats = sres;
        return FPM_OK;
    }

    // a plan whose buffers are carved from the scratch array (nothing of
    // it is ever freed); the persistent, device-scheduled pipeline with
    // plain launches
    fpm_plan p;
    p.ix = ix;
    p.max_q = kNaMaxQueries;
    p.max_bytes = query_bytes;
    p.metric = metric;
    p.k = k;
    p.opt = o;
    p.opt.schedule = o.schedule == FPM_SCHED_BRUTE ? FPM_SCHED_BRUTE : FPM_SCHED_BATCHED;
    p.stream = (hipStream_t)hip_stream;
    p.kind = p.opt.schedule == FPM_SCHED_BRUTE ? kAll : ix->kind;
    const int key_width = ix->bits == 16 && ix->variant != FPM_COUNT ? 16 : 32;
    p.mx_width = p.kind != kAll && mx_ok && o.filter_unit == FPM_UNIT_MATRIX ? key_width : 0;
    if (p.mx_width && !(opt && opt->waves_per_cu))
        p.opt.waves_per_cu = 28;
    uint8_t *b = nd.base;
    StrSet &Q = p.q;
    Q.cap_n = kNaMaxQueries;
    Q.cap_bytes = query_bytes;
    Q.str_cap = kNa.str_cap;
    Q.len = (uint32_t *)(b + kNa.len);
    Q.perm = (uint32_t *)(b + kNa.perm);
    Q.soff = (uint32_t *)(b + kNa.soff);
    Q.slen = b + kNa.slen;
    Q.off = (uint32_t *)(b + kNa.off);
    Q.bdw = (uint32_t *)(b + kNa.bdw);
    Q.str = (uint32_t *)(b + kNa.str);
    Q.key = b + kNa.key;
    p.scratch = (uint32_t *)(b + kNa.radix);
    p.pairs = (PairRec *)(b + kNa.pairs);
    p.ctr = (DevCounters *)(b + kNa.ctr);
    p.keys = (uint64_t *)(b + kNa.keys);
    p.tmp = (uint64_t *)(b + kNa.tmp);
    p.qexp = p.mx_width ? b + kNa.qexp : nullptr;
    // the sort's last pass writes the triples straight into the caller's
    // buffer: at most min(out_cap, kNaMaxMatches) of them
    p.triples = (uint32_t *)d_out;
    p.cap = std::min<uint64_t>(out_cap, kNaMaxMatches);
    p.persistent_blocks = std::max(1, nd.cus * (int)p.opt.waves_per_cu / 4);

    st = enqueue_prep(&p, d_qbytes, d_qoffsets, n_queries, false);
    if (!st)
        st = enqueue_kernel(&p, false);
    if (st)
        return st;
    enqueue_post(&p, n_queries);
    DevCounters c;
    HIPCHK(hipMemcpyAsync(&c, p.ctr, offsetof(DevCounters, counters), hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    if (c.err)
        return fail(FPM_EINVAL, "query batch: %s",
                    (c.err & 2) ? "offsets decrease"
                                : (c.err & 1) ? "a string is longer than 255" : "more bytes than query_bytes");
    *n_out = c.n_out;
    if (c.n_out > kNaMaxMatches)
        return fail(FPM_ENOMEM, "%llu matches exceed the allocation-free limit of %llu (use a plan)",
                    (unsigned long long)c.n_out, (unsigned long long)kNaMaxMatches);
    if (c.n_out > out_cap)
        return fail(FPM_EINVAL, "%llu matches do not fit out_cap = %llu", (unsigned long long)c.n_out,
                    (unsigned long long)out_cap);
    sres.pairs_examined = c.examined;
    sres.survivors = c.survivors;
    sres.matches = c.n_out;
    sres.verify_cells = c.cells;
    sres.pairs_filtered = p.kind == kAll ? 0 : c.examined - std::min(c.pruned, c.examined);
    sres.work_items = c.n_items;
    sres.filter_unit = p.kind == kAll ? FPM_UNIT_AUTO : p.mx_width ? FPM_UNIT_MATRIX : FPM_UNIT_VALU;
    if (stats)
        *stats = sres;
    return FPM_OK;
}

// Temporary device copy of host strings, sorted and fingerprinted.
struct TmpSet {
    StrSet S;
    uint8_t *b = nullptr;
    uint64_t *o = nullptr;
    uint32_t *scratch = nullptr, *err = nullptr;
    hipStream_t s = nullptr;
    ~TmpSet()
    {
        S.release();
        dfree(b);
        dfree(o);
        dfree(scratch);
        dfree(err);
        if (s)
            (void)hipStreamDestroy(s);
    }
    fpm_status make(const fpm_index *ix, const uint8_t *bytes, const uint64_t *offsets, uint32_t n, bool fp_orig)
    {
        const uint64_t nbytes = offsets[n];
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) || (e = dalloc(&b, nbytes + 4)) ||
            (e = dalloc(&o, (size_t)n + 1)) || (e = dalloc(&scratch, kRadixScratch)) || (e = dalloc(&err, 1)) ||
            (e = S.alloc(n, nbytes + 4, ix->kind, fp_orig, true, false)))
            return hip_fail(e, "temporary string set");
        if (nbytes)
            (void)hipMemcpyAsync(b, bytes, nbytes, hipMemcpyHostToDevice, s);
        (void)hipMemcpyAsync(o, offsets, sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s);
        launch_zero(err, 1, s);
        prep_strings(S, b, o, n, nbytes, ix->d_map, ix->variant, ix->bits, ix->kind, true, false, err, scratch, s);
        launch_invert(S.perm, n, S.inv, s);
        uint32_t h_err = 0;
        if ((e = hipMemcpyAsync(&h_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) ||
            (e = hipStreamSynchronize(s)))
            return hip_fail(e, "temporary string set");
        if (h_err)  // the host checks leave only a layout overflow
            return fail(FPM_EDEVICE, "temporary string set: padded layout failed (flags %u)", h_err);
        return FPM_OK;
    }
};

fpm_status fpm_fingerprints(const fpm_index *ix, const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                            uint32_t *out)
{
    g_last_error.clear();
    if (!ix || (n && !out))
        return fail(FPM_EINVAL, "null pointer");
    fpm_status st = check_csr(bytes, offsets, n, "strings");
    if (st || n == 0)
        return st;
    TmpSet t;
    st = t.make(ix, bytes, offsets, n, true);
    if (st)
        return st;
    HIPCHK(hipMemcpyAsync(out, t.S.fp_orig, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, t.s));
    HIPCHK(hipStreamSynchronize(t.s));
    return FPM_OK;
}

fpm_status fpm_verify_pairs(const fpm_index *ix, const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                            const uint32_t *pairs, uint64_t n_pairs, fpm_metric metric, uint32_t k, uint32_t *dist_out)
{
    g_last_error.clear();
    if (!ix || (n_pairs && (!pairs || !dist_out)))
        return fail(FPM_EINVAL, "null pointer");
    if (metric != FPM_HAM && metric != FPM_LEV)
        return fail(FPM_EINVAL, "unknown metric");
    if (k < 1 || k > (uint32_t)kMaxK)
        return fail(FPM_EUNSUPPORTED, "k must be 1 .. %d", kMaxK);
    fpm_status st = check_csr(qbytes, qoffsets, n_queries, "queries");
    if (st || n_pairs == 0)
        return st;
    for (uint64_t i = 0; i < n_pairs; ++i)
        if (pairs[2 * i] >= n_queries || pairs[2 * i + 1] >= ix->n)
            return fail(FPM_EINVAL, "pair %llu out of range", (unsigned long long)i);
    TmpSet t;
    st = t.make(ix, qbytes, qoffsets, n_queries, false);
    if (st)
        return st;
    uint32_t *d_pairs = nullptr, *d_dist = nullptr;
    hipError_t e;
    if ((e = dalloc(&d_pairs, 2 * n_pairs)) || (e = dalloc(&d_dist, n_pairs))) {
        dfree(d_pairs);
        return hip_fail(e, "verify alloc");
    }
    (void)hipMemcpyAsync(d_pairs, pairs, sizeof(uint32_t) * 2 * n_pairs, hipMemcpyHostToDevice, t.s);
    e = launch_verify_pairs(t.S.view(), t.S.inv, ix->words.view(), ix->words.inv, d_pairs, n_pairs, metric, k, d_dist,
                            t.s);
    if (!e)
        e = hipMemcpyAsync(dist_out, d_dist, sizeof(uint32_t) * n_pairs, hipMemcpyDeviceToHost, t.s);
    if (!e)
        e = hipStreamSynchronize(t.s);
    dfree(d_pairs);
    dfree(d_dist);
    if (e)
        return hip_fail(e, "fpm_verify_pairs");
    return FPM_OK;
}

fpm_status fpm_autotune(const fpm_index *ix, const uint8_t *d_qbytes, const uint64_t *d_qoffsets, uint32_t n_queries,
                        uint64_t query_bytes, fpm_metric metric, uint32_t k, uint32_t repeats, fpm_options *best,
                        float *timings_out, uint32_t max_timings, uint32_t *n_timings)
{
    g_last_error.clear();
    if (!ix || !best)
        return fail(FPM_EINVAL, "null pointer");
    static const uint32_t qts[] = {16, 32, 64, 128, 256};
    static const uint32_t slabs[] = {512, 1024, 2048, 4096, 8192, 16384};
    static const uint32_t tails[] = {10, 25, 40};
    if (repeats == 0)
        repeats = 3;
    fpm_options base = *best;
    if (!base.tail_split)
        base.tail_split = 100;
    float best_ms = 1e30f;
    uint32_t nt = 0;
    std::vector<std::pair<float, fpm_options>> seen;
    // time one configuration; the fastest so far goes to *best
    auto trial = [&](fpm_options o, uint32_t repeats) -> fpm_status {
        o.schedule = FPM_SCHED_BATCHED;
        if (!o.use_graph)
            o.use_graph = 1;
        fpm_plan *p = nullptr;
        fpm_status st = plan_create(ix, n_queries, query_bytes, metric, k, &o, nullptr, false, &p);
        if (st)
            return st;
        float tot = 0.f;
        for (uint32_t r = 0; r <= repeats && !st; ++r) {
            st = fpm_plan_run(p, d_qbytes, d_qoffsets, n_queries);
            fpm_stats s;
            if (!st)
                st = fpm_plan_result(p, nullptr, nullptr, &s);
            if (!st && r > 0)
                tot += s.ms;
        }
        if (!st)
            o.match_capacity = (uint32_t)std::min<uint64_t>(p->cap, 0xFFFFFFFFu);
        plan_free(p);
        if (st)
            return st;
        const float ms = tot / repeats;
        seen.emplace_back(ms, o);
        if (timings_out && nt < max_timings) {
            timings_out[5 * nt + 0] = (float)o.queries_per_item;
            timings_out[5 * nt + 1] = (float)o.slab;
            timings_out[5 * nt + 2] = (float)o.bucket_order;
            timings_out[5 * nt + 3] = (float)o.tail_split;
            timings_out[5 * nt + 4] = ms;
        }
        ++nt;
        if (ms < best_ms) {
            best_ms = ms;
            *best = o;
        }
        return FPM_OK;
    };
    for (uint32_t order = 0; order < 2; ++order) {
        for (uint32_t qt : qts) {
            for (uint32_t sl : slabs) {
                fpm_options o = base;
                o.queries_per_item = qt;
                o.slab = sl;
                o.bucket_order = order;
                if (fpm_status st = trial(o, repeats))
                    return st;
            }
        }
    }
    const fpm_options grid_best = *best;
    for (uint32_t tl : tails) {
        if (tl == grid_best.tail_split)
            continue;
        fpm_options o = grid_best;
        o.tail_split = tl;
        if (fpm_status st = trial(o, repeats))
            return st;
    }
    // the short timings above are a few percent noisy: time the four fastest
    // again, longer, and keep the fastest of those
    std::vector<std::pair<float, fpm_options>> top(seen);
    std::sort(top.begin(), top.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    top.resize(std::min<size_t>(top.size(), 4));
    best_ms = 1e30f;
    for (const auto &c : top)
        if (fpm_status st = trial(c.second, std::max<uint32_t>(8, 4 * repeats)))
            return st;
    if (n_timings)
        *n_timings = std::min(nt, max_timings);
    return FPM_OK;
}

}  // extern "C"
