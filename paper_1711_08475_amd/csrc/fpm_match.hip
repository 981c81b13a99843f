// fpm_match.hip -- the matching hot path: fingerprint filter (Section 3.3,
// Eq. 1), survivor compaction and exact verification, fused in one kernel.
//
// Work decomposition.  Queries and words are sorted by length, so a pair of
// length buckets (query length m, word length L) is length-compatible when
// L = m (Hamming; a Hamming distance between unequal lengths is infinite) or
// |L - m| <= k (Levenshtein >= |L - m|).  Each compatible pair of buckets is
// cut into work items: a tile of up to `qtile` queries of length m times a
// slab of up to `slab` words of length L.  A work item belongs to one wave.
// The persistent launch gives wave w item w first, then hands out the rest
// through eight striped atomic counters (no single contended address, no
// burst of atomics at start-up), and each wave's issue priority follows its
// item's position in the list so that items finish about in list order.
//
// Per work item, per 128 dictionary words (two per lane, two independent
// mask chains) and per 32 queries (two groups of 16 filter keys,
// wave-uniform, loaded into scalar registers):
//   t   = popcount(kq ^ kw) - (2k + 1)   one v_xor, one v_bcnt with accumulator
//   msk = (msk << 1) | (t >> 31)         one v_alignbit: sign bit = F_D <= 2k
// i.e. three vector instructions per (query, word) pair (other key
// families: position fields 8, bigrams 3 against 4k, the asymmetric bound 3
// or 4, 64-bit keys 5 or 6).  On the matrix cores (16- and 32-bit
// popcount-of-XOR keys, the matrix-filter section below) a pass is instead
// 64 queries x 64 words (32-bit keys: x 32) computed as an int8 matrix
// product whose sign bits land in masks of the same layout, one
// v_alignbit per 64 pairs.  Under the asymmetric bound the query and word
// blocks are ordered by key popcount, and items and 32 x 128 passes whose
// popcount ranges cannot meet are skipped.  Each of the lane's
// two 32-bit survivor masks is then appended to a per-wave queue in LDS:
// each lane with survivors reserves its range with one LDS atomic add on
// the wave's queue counter (the LDS unit serialises the lanes, the VALU
// computes no prefix sum; entry order does not matter); when 32 queries'
// survivors would not fit, the two halves are appended one after the other
// with drains in between (every pair survives, e.g., in the brute-force
// form).  Every time the queue holds 64 entries the wave pops 64 and
// verifies them, one per lane, so the verifier always runs on full waves.
// Matches leave through one atomic per flush of a per-wave LDS staging
// buffer.
//
// Verifiers (k-bounded, exact below k+1):
//   Ham:   word-parallel mismatch count over 4-byte groups, exit above k;
//   Lev 1: equal lengths -> Ham <= 1; lengths differing by one -> the shorter
//          string s and longer t are one deletion apart iff the last
//          position where s[j] != t[j+1] lies before the first position where
//          s[j] != t[j]; both positions come from XORs of 4-byte groups
//          (t shifted by one byte with v_alignbyte) and ctz / clz;
//   Lev k>=2: the 2k+1 diagonal band of the edit-distance table (Ukkonen's
//          cut-off, as the paper's 2k+1 strip), two band rows in registers.
#include "fpm_internal.hpp"

namespace fpm {

namespace {

constexpr int kWaves = 4;                 // waves per block, each independent
constexpr int kChunk = 16;                // filter keys per scalar load; a pass covers 2 * kChunk queries
constexpr int kQueueCap = 64 * kChunk + 64;  // entries per wave: < 64 left + one half pass
// Matches are staged per wave in LDS and leave through one atomic per flush;
// a flush happens once more than kOutFlush are staged, so a drain (<= 64
// new matches) always fits.  Queue + staging + queue counter = 5116 bytes
// per wave; with the block's exhausted-stripe mask 20,472 bytes per block,
// so eight blocks fit the 160 KB of LDS of a compute unit.
constexpr int kOutCap = 95;
constexpr int kOutFlush = kOutCap - 64;

// -------------------------------------------------------------- filters
// test() returns a value whose sign bit is set iff the pair survives the
// family's rule (F_D <= 2k for the paper's fingerprints); `neg` holds
// filter_neg<KIND, K>() (-(2k + 1) for those).
template <int KIND>
struct Filter;

template <>
struct Filter<kPop32> {
    using Key = uint32_t;
    static __device__ __forceinline__ uint32_t test(Key q, Key w, uint32_t neg)
    {
        return (uint32_t)__builtin_popcount(q ^ w) + neg;
    }
};

template <>
struct Filter<kPop64> {
    using Key = uint64_t;
    static __device__ __forceinline__ uint32_t test(Key q, Key w, uint32_t neg)
    {
        const uint64_t x = q ^ w;
        return (uint32_t)__builtin_popcount((uint32_t)x) + (uint32_t)__builtin_popcount((uint32_t)(x >> 32)) + neg;
    }
};

// position fingerprints: count 3-bit fields that differ (a field differs
// iff the OR of its three XOR bits is set, gathered at the field's low bit)
// plus the differing occurrence bits.
template <>
struct Filter<kPos16> {
    using Key = uint32_t;
    static __device__ __forceinline__ uint32_t test(Key q, Key w, uint32_t neg)
    {
        const uint32_t x = q ^ w;
        const uint32_t y = x | (x >> 1) | (x >> 2);
        return (uint32_t)__builtin_popcount((y & 0x1249u) | (x & 0x8000u)) + neg;
    }
};

template <>
struct Filter<kPos32> {
    using Key = uint32_t;
    static __device__ __forceinline__ uint32_t test(Key q, Key w, uint32_t neg)
    {
        const uint32_t x = q ^ w;
        const uint32_t y = x | (x >> 1) | (x >> 2);
        return (uint32_t)__builtin_popcount((y & 0x09249249u) | (x & 0xC0000000u)) + neg;
    }
};

template <>
struct Filter<kAll> {
    using Key = uint32_t;
    static __device__ __forceinline__ uint32_t test(Key, Key, uint32_t) { return 0x80000000u; }
};

// Asymmetric bound, thermometer form: the key's upper half holds the
// thermometer code of the popcount of its lower half, so the XOR weight is
// F_D + |pq - pw| = 2 max(e(q, w), e(w, q)) and the F_D <= 2k test applies.
template <>
struct Filter<kTherm32> : Filter<kPop32> {
};

// Bigram fingerprints: the same XOR popcount, against 4k (filter_neg).
template <>
struct Filter<kQgram32> : Filter<kPop32> {
};

// The popcount-ordered variants test pairs exactly as their base kinds.
template <>
struct Filter<kPop32P> : Filter<kPop32> {
};
template <>
struct Filter<kPop64P> : Filter<kPop64> {
};
template <>
struct Filter<kQgram32P> : Filter<kPop32> {
};

// Combined fingerprints: each word's XOR popcount against 2k; the AND of the
// two tests has its sign bit set iff both parts pass.
template <>
struct Filter<kCombo64> {
    using Key = uint64_t;
    static __device__ __forceinline__ uint32_t test(Key q, Key w, uint32_t neg)
    {
        const uint64_t x = q ^ w;
        return ((uint32_t)__builtin_popcount((uint32_t)x) + neg) &
               ((uint32_t)__builtin_popcount((uint32_t)(x >> 32)) + neg);
    }
};

// Asymmetric bound on full-width keys: with c = popc(q & w) the larger
// excess is max(pq, pw) - c, and it is <= k iff
// popc(~(q & w)) + max(pq, pw) - (width + k + 1) < 0.  Each side's popcount
// plus `neg` = -(width + k + 1) is computed once per query (scalar) and once
// per word (vector), so a pair costs a NAND, a max and the popcount that
// accumulates onto the max.  The empty asm statements keep the compiler
// from pulling the shared bias out of the max (which would add one more
// instruction per pair).
__device__ __forceinline__ uint32_t opaque_v(uint32_t x)
{
    asm("" : "+v"(x));
    return x;
}
__device__ __forceinline__ uint32_t opaque_s(uint32_t x)
{
    asm("" : "+s"(x));
    return x;
}
template <typename T>
__device__ __forceinline__ T *opaque_ptr(T *p)
{
    asm("" : "+s"(p));
    return p;
}

template <>
struct Filter<kAsym32> {
    using Key = uint32_t;
    static __device__ __forceinline__ uint32_t side_w(Key w, uint32_t neg)
    {
        return opaque_v((uint32_t)__builtin_popcount(w) + neg);
    }
    static __device__ __forceinline__ uint32_t side_q(Key q, uint32_t neg)
    {
        return opaque_s((uint32_t)__builtin_popcount(q) + neg);
    }
    static __device__ __forceinline__ uint32_t test(Key q, uint32_t sq, Key w, uint32_t sw)
    {
        return (uint32_t)__builtin_popcount(~(q & w)) + (uint32_t)max((int)sq, (int)sw);
    }
};

template <>
struct Filter<kAsym64> {
    using Key = uint64_t;
    static __device__ __forceinline__ uint32_t side_w(Key w, uint32_t neg)
    {
        return opaque_v((uint32_t)__popcll(w) + neg);
    }
    static __device__ __forceinline__ uint32_t side_q(Key q, uint32_t neg)
    {
        return opaque_s((uint32_t)__popcll(q) + neg);
    }
    static __device__ __forceinline__ uint32_t test(Key q, uint32_t sq, Key w, uint32_t sw)
    {
        const uint64_t x = ~(q & w);
        return (uint32_t)__builtin_popcount((uint32_t)(x >> 32)) +
               ((uint32_t)__builtin_popcount((uint32_t)x) + (uint32_t)max((int)sq, (int)sw));
    }
};

// -(threshold + 1) of each key family's test.
template <int KIND, int K>
__host__ __device__ constexpr uint32_t filter_neg()
{
    return KIND == kAsym32    ? 0u - (32u + K + 1u)
           : KIND == kAsym64  ? 0u - (64u + K + 1u)
           : (KIND == kQgram32 || KIND == kQgram32P) ? 0u - (4u * K + 1u)
                              : 0u - (2u * K + 1u);
}

// Families whose blocks are ordered by key popcount, so that a tile spans
// [pop(first), pop(last)] and a pair whose key popcounts differ by more than
// pop_gap cannot survive: the asymmetric bound's (e(q, w) - e(w, q) =
// pq - pw: 2k in thermometer units, k otherwise) and the paper's rule on
// popcount-ordered blocks (F_D = popc(kq ^ kw) >= |pq - pw|: the threshold,
// 2k or 4k for bigrams).
template <int KIND>
__host__ __device__ constexpr bool pop_skip()
{
    return KIND == kTherm32 || KIND == kAsym32 || KIND == kAsym64 || KIND == kPop32P || KIND == kPop64P ||
           KIND == kQgram32P;
}

template <int KIND>
__host__ __device__ constexpr bool side_values()
{
    return KIND == kAsym32 || KIND == kAsym64;
}

// One query against the lane's two words: the test's sign bit goes into bit
// 0 of each mask (older bits move up).  sa / sb: the words' side values.
template <int KIND>
__device__ __forceinline__ void filter_step(typename Filter<KIND>::Key q, typename Filter<KIND>::Key wa,
                                            typename Filter<KIND>::Key wb, uint32_t sa, uint32_t sb, uint32_t neg,
                                            uint32_t &ma, uint32_t &mb)
{
    using F = Filter<KIND>;
    if constexpr (side_values<KIND>()) {
        const uint32_t sq = F::side_q(q, neg);
        ma = __builtin_amdgcn_alignbit(ma, F::test(q, sq, wa, sa), 31);
        mb = __builtin_amdgcn_alignbit(mb, F::test(q, sq, wb, sb), 31);
    } else {
        ma = __builtin_amdgcn_alignbit(ma, F::test(q, wa, neg), 31);
        mb = __builtin_amdgcn_alignbit(mb, F::test(q, wb, neg), 31);
    }
}

template <int KIND, int K>
__host__ __device__ constexpr uint32_t pop_gap()
{
    return KIND == kQgram32P                                          ? 4u * K
           : (KIND == kTherm32 || KIND == kPop32P || KIND == kPop64P) ? 2u * K
                                                                      : (uint32_t)K;
}

__device__ __forceinline__ uint32_t key_pop(uint32_t v) { return (uint32_t)__builtin_popcount(v); }
__device__ __forceinline__ uint32_t key_pop(uint64_t v) { return (uint32_t)__popcll(v); }

// Wave-uniform copy of lane l's key (l uniform).
__device__ __forceinline__ uint32_t lane_key(uint32_t v, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint64_t lane_key(uint64_t v, uint32_t l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l);
    return ((uint64_t)hi << 32) | lo;
}

// Two popcount ranges that no pair can bridge.
__device__ __forceinline__ bool pop_apart(uint32_t alo, uint32_t ahi, uint32_t blo, uint32_t bhi, uint32_t gap)
{
    return alo > bhi + gap || blo > ahi + gap;
}

// ------------------------------------------------------------ verifiers
// All verifiers see wave-uniform lengths (every entry of a drain comes from
// one work item, i.e. one pair of length buckets), so loop trip counts and
// branches on lengths are uniform; strings are read from their padded slots
// 16 bytes at a time.

// Dwords g0 .. g0+D-1 of a string (load_raw), then bytes at positions >=
// len cleared (mask_tail).  Every layout kernel writes whole slots, zero
// beyond the string's length, so only a dword past the slot needs the mask:
// the Lev k = 1 test's one extra dword of the longer string, which may lie in
// the next slot (the string buffers' tail slack covers a read past the last
// one).  The verifiers issue every load of a step before any mask (one
// memory round trip); len is wave-uniform in the match kernel, so the masks
// are scalar.
template <int D>
__device__ __forceinline__ void load_raw(const uint32_t *p, uint32_t g0, uint32_t (&v)[D])
{
#pragma unroll
    for (int t = 0; t < D; ++t)
        v[t] = p[g0 + t];
}

template <int D>
__device__ __forceinline__ void mask_tail(uint32_t g0, uint32_t len, uint32_t (&v)[D])
{
#pragma unroll
    for (int t = 0; t < D; ++t) {
        // written with selects only (no min / max), so a uniform length keeps
        // the mask in scalar registers
        const int rem = (int)len - 4 * (int)(g0 + t);
        const uint32_t part = (1u << (8u * ((uint32_t)rem & 3u))) - 1u;
        const uint32_t m = rem >= 4 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : part);
        v[t] &= m;
    }
}

// number of nonzero bytes of x
__device__ __forceinline__ uint32_t nz_bytes(uint32_t x)
{
    return (uint32_t)__builtin_popcount((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

// Dwords g0 .. g0+D-1 of two strings of one length lie inside both slots.
template <int D>
__device__ __forceinline__ uint32_t ham_dwords(const uint32_t *a, const uint32_t *b, uint32_t g0)
{
    uint32_t A[D], B[D];
    load_raw<D>(a, g0, A);
    load_raw<D>(b, g0, B);
    uint32_t d = 0;
#pragma unroll
    for (int t = 0; t < D; ++t)
        d += nz_bytes(A[t] ^ B[t]);
    return d;
}

// Hamming distance of two strings of length m, capped at K + 1.
template <int K>
__device__ __forceinline__ uint32_t verify_ham(const uint32_t *a, const uint32_t *b, uint32_t m)
{
    uint32_t d;
    if (m <= 4) {
        d = ham_dwords<1>(a, b, 0);
    } else if (m <= 8) {
        d = ham_dwords<2>(a, b, 0);
    } else {
        d = 0;
        const uint32_t nch = (m + 15) >> 4;
        for (uint32_t c = 0; c < nch; ++c) {
            d += ham_dwords<4>(a, b, 4 * c);
            if (!__any(d <= (uint32_t)K))
                break;
        }
    }
    return min(d, (uint32_t)K + 1);
}

// One group of D dwords of the Lev k = 1 test for lengths m and n = m + 1
// (a shorter): first_a tracks the first j with a[j] != b[j] (clamped to m),
// last_b the last j with a[j] != b[j + 1].  Dwords g0 .. g0+D-1 lie inside
// both slots (slot_dwords(m + 1) >= slot_dwords(m)); b's dword g0 + D may
// not, and is masked.
template <int D>
__device__ __forceinline__ void lev1_dwords(const uint32_t *a, const uint32_t *b, uint32_t g0, uint32_t m,
                                            uint32_t &first_a, int &last_b)
{
    uint32_t A[D], B[D + 1];
    load_raw<D>(a, g0, A);
    load_raw<D + 1>(b, g0, B);
    uint32_t (&Bx)[1] = *reinterpret_cast<uint32_t (*)[1]>(&B[D]);
    mask_tail<1>(g0 + D, m + 1, Bx);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const uint32_t xa = A[t] ^ B[t];
        const uint32_t xb = A[t] ^ __builtin_amdgcn_alignbyte(B[t + 1], B[t], 1);
        const uint32_t pos = 4 * (g0 + t);
        if (first_a == m && xa != 0u)
            first_a = min(pos + ((uint32_t)__builtin_ctz(xa) >> 3), m);
        if (xb != 0u)
            last_b = (int)(pos + ((31u - (uint32_t)__builtin_clz(xb)) >> 3));
    }
}

// Levenshtein distance <= 1 test.  Equal lengths: Hamming <= 1.  Lengths m
// and m + 1: with a the shorter string and b the longer one, b becomes a by
// deleting one symbol iff every position j with a[j] != b[j + 1] lies before
// the first position with a[j] != b[j] (then delete b at that position).
__device__ __forceinline__ uint32_t verify_lev1(const uint32_t *a, uint32_t m, const uint32_t *b, uint32_t n)
{
    if (m == n)
        return verify_ham<1>(a, b, m);
    if (m > n) {
        const uint32_t *t = a;
        a = b;
        b = t;
        const uint32_t u = m;
        m = n;
        n = u;
    }
    if (n - m != 1)
        return 2;
    uint32_t first_a = m;
    int last_b = -1;
    if (m <= 4) {
        lev1_dwords<1>(a, b, 0, m, first_a, last_b);
    } else if (m <= 8) {
        lev1_dwords<2>(a, b, 0, m, first_a, last_b);
    } else {
        const uint32_t nch = (m + 15) >> 4;
        for (uint32_t c = 0; c < nch; ++c) {
            lev1_dwords<4>(a, b, 4 * c, m, first_a, last_b);
            if (!__any(last_b < (int)first_a))
                break;
        }
    }
    return last_b < (int)first_a ? 1u : 2u;
}

// Bytes of a padded string in order, one dword load per four bytes; indices
// below zero or past the slot read as zero.  The read schedule depends only
// on the (uniform) index.
struct ByteStream {
    const uint32_t *p;
    uint32_t sw;
    int idx;
    uint32_t cur;
    __device__ __forceinline__ uint32_t next()
    {
        const int i = idx++;
        if (i < 0)
            return 0u;
        if ((i & 3) == 0)
            cur = ((uint32_t)i >> 2) < sw ? p[i >> 2] : 0u;
        return (cur >> (8 * (i & 3))) & 0xFFu;
    }
};

// Banded edit distance (Ukkonen's cut-off: only |j - i| <= K matters when
// the distance is at most K), cells outside the band held at K + 1, the
// result capped at K + 1.  Row i keeps cells
// j = i - K .. i + K; `win` holds the symbols b[j - 1] those cells compare,
// byte t for j = i + t - K.
template <int K>
__device__ __forceinline__ uint32_t verify_lev_band(const uint32_t *a, uint32_t m, const uint32_t *b, uint32_t n)
{
    const int gap = (int)n - (int)m;
    if (gap > K || gap < -K)
        return K + 1;
    constexpr uint32_t INF = K + 1;
    constexpr int W = 2 * K + 1;
    uint32_t prev[W], cur[W];
#pragma unroll
    for (int t = 0; t < W; ++t) {
        const int j = t - K;
        prev[t] = (j >= 0 && j <= (int)n) ? min((uint32_t)j, INF) : INF;
    }
    ByteStream as{a, (m + 3) >> 2, 0, 0u};
    ByteStream bs{b, (n + 3) >> 2, -K, 0u};  // row 1 compares b[-K .. K] (1-indexed j = 1 - K .. 1 + K)
    uint64_t win = 0;
#pragma unroll
    for (int t = 0; t < W; ++t)
        win |= (uint64_t)bs.next() << (8 * t);
    for (uint32_t i = 1; i <= m; ++i) {
        const uint32_t ai = as.next();
        uint32_t rowmin = INF;
#pragma unroll
        for (int t = 0; t < W; ++t) {
            const int j = (int)i + t - K;
            uint32_t v;
            if (j < 0 || j > (int)n) {
                v = INF;
            } else if (j == 0) {
                v = min(i, INF);
            } else {
                // a byte field extract lets the compare read the byte in place
                const uint32_t bj =
                    __builtin_amdgcn_ubfe(t < 4 ? (uint32_t)win : (uint32_t)(win >> 32), 8u * (uint32_t)(t & 3), 8u);
                // no clamp at INF: cells outside the band enter as INF, so any
                // value computed through them exceeds k, and values <= k are
                // exact (Ukkonen's band); the result is clamped at the end
                const uint32_t diag = prev[t] + (ai != bj ? 1u : 0u);
                const uint32_t up = (t + 1 < W) ? prev[t + 1] + 1u : INF;
                const uint32_t left = (t >= 1) ? cur[t - 1] + 1u : INF;
                v = min(min(diag, up), left);
            }
            cur[t] = v;
            rowmin = min(rowmin, v);
        }
        if (!__any(rowmin <= (uint32_t)K))
            return K + 1;
#pragma unroll
        for (int t = 0; t < W; ++t)
            prev[t] = cur[t];
        win = (win >> 8) | ((uint64_t)bs.next() << (8 * (W - 1)));
    }
    return min(prev[gap + K], INF);
}

template <int METRIC, int K>
__device__ __forceinline__ uint32_t verify(const uint32_t *a, uint32_t m, const uint32_t *b, uint32_t n)
{
    if (METRIC == 0)
        return m == n ? verify_ham<K>(a, b, m) : K + 1;
    if (K == 1)
        return verify_lev1(a, m, b, n);
    return verify_lev_band<K>(a, m, b, n);
}

// Wave-uniform, read-only data (work list, query keys) is read through the
// constant address space so that it is fetched with scalar loads into SGPRs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)(p);
}

// The match kernel's arguments, read from the kernel-argument segment where
// they are used (the match-list flushes and the block epilogue, a few times
// per wave): the empty asm makes each use a fresh scalar load, so that these
// values hold no scalar registers across the loops.  The vector-filter
// kernel has 80 scalar registers at eight waves per SIMD.
__device__ __forceinline__ cptr<MatchArgs> kargs()
{
    uint64_t p = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return (cptr<MatchArgs>)p;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---------------------------------------------------------- work items

struct Item {
    uint32_t qs, qn;        // sorted query range
    uint32_t ds, de;        // sorted dictionary range
    uint32_t m, L;          // query length, word length
    uint32_t qsw, dsw;      // slot sizes in dwords
    const uint32_t *qstr, *dstr;    // slots of the item's first query / word
    const uint32_t *qperm, *dperm;  // caller indices from the item's first query / word on
};

__device__ __forceinline__ Item decode_item(const MatchArgs &a, uint32_t item, uint32_t n_pairs)
{
    // last pair whose item_base <= item (uniform binary search)
    const cptr<PairRec> pairs = as_const(a.wl.pairs);
    uint32_t lo = 0, hi = n_pairs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pairs[mid].item_base <= item)
            lo = mid;
        else
            hi = mid;
    }
    const uint32_t base = pairs[lo].item_base, qbase = pairs[lo].qbase, nq = pairs[lo].nq;
    const uint32_t dbase = pairs[lo].dbase, nd = pairs[lo].nd, tiles_d = pairs[lo].tiles_d;
    const uint32_t qtile = pairs[lo].qtile, slab = pairs[lo].slab;
    const uint32_t t = item - base;
    const uint32_t tq = t / tiles_d, td = t - tq * tiles_d;
    Item it;
    it.qs = qbase + tq * qtile;
    it.qn = min(qtile, qbase + nq - it.qs);
    it.ds = dbase + td * slab;
    it.de = min(it.ds + slab, dbase + nd);
    it.m = pairs[lo].qlen;
    it.L = pairs[lo].dlen;
    it.qstr = a.q.str + as_const(a.q.soff)[it.qs];
    it.dstr = a.d.str + as_const(a.d.soff)[it.ds];
    it.qperm = a.q.perm + it.qs;
    it.dperm = a.d.perm + it.ds;
    it.qsw = slot_dwords(it.m);
    it.dsw = slot_dwords(it.L);
    return it;
}

// Queue entries are item-relative: query offset in the tile (10 bits) and
// word offset in the slab (22 bits).
constexpr uint32_t kWordBits = 22;

// Write the staged matches of a wave to the global match list.
__device__ __forceinline__ void flush(const MatchArgs &a, const uint64_t *out, uint32_t &ocount, uint32_t lane)
{
    __builtin_amdgcn_wave_barrier();
    const cptr<MatchArgs> A = kargs();
    unsigned long long base = 0;
    if (lane == 0)
        base = atomicAdd((unsigned long long *)A->ctr.n_out, (unsigned long long)ocount);
    base = __shfl(base, 0);
    for (uint32_t i = lane; i < ocount; i += 64) {
        const uint64_t idx = base + i;
        if (idx < A->out_cap)
            A->out_keys[idx] = out[i];
    }
    __builtin_amdgcn_wave_barrier();
    ocount = 0;
}

// Pop `nact` (<= 64) entries from the wave queue, verify one per lane and
// stage the matches.
template <int METRIC, int K>
__device__ __forceinline__ void drain(const MatchArgs &a, const Item &it, const uint32_t *queue, uint32_t &qlen,
                                      uint32_t nact, uint32_t lane, uint64_t *out, uint32_t &ocount)
{
    __builtin_amdgcn_wave_barrier();
    const bool act = lane < nact;
    const uint32_t ent = act ? queue[qlen - nact + lane] : 0u;
    __builtin_amdgcn_wave_barrier();
    qlen -= nact;
    const uint32_t tq = ent >> kWordBits, te = ent & ((1u << kWordBits) - 1u);
    uint32_t d = K + 1;
    if (act) {
        // 32-bit slot offsets (unsigned: no sign extension into the address)
        const uint32_t qo = (uint32_t)__umul24(tq, it.qsw), wo = (uint32_t)__umul24(te, it.dsw);
        d = a.survivors_only ? 0u : verify<METRIC, K>(it.qstr + qo, it.m, it.dstr + wo, it.L);
    }
    const bool ok = act && d <= (uint32_t)K;
    const uint64_t mm = __ballot(ok);
    if (mm) {
        if (ok) {
            // both caller indices in one memory round trip
            const uint32_t qi = it.qperm[tq], wi = it.dperm[te];
            out[ocount + lanes_below(mm)] = ((uint64_t)qi << (a.wbits + 2)) | ((uint64_t)wi << 2) | d;
        }
        ocount += (uint32_t)__popcll(mm);
        if (ocount > (uint32_t)kOutFlush)
            flush(a, out, ocount, lane);
    }
}

// Append one lane's survivor mask to the wave queue: bit b is the entry
// ent0 + (b << kWordBits).  Each lane with survivors reserves its range with
// one LDS atomic on the wave's counter.  The caller drains the queue, 64
// entries at a time, after the pass's masks are in (one drain site per pass
// keeps the verifier's registers out of the filter loop).  When the wave's
// survivors would overflow the queue the mask goes in as two 16-bit halves
// with drains in between.
template <int METRIC, int K>
__device__ __forceinline__ void append(const MatchArgs &a, const Item &it, uint32_t *queue, uint32_t *qcnt,
                                       uint32_t &qlen, uint32_t msk, uint32_t ent0, uint32_t lane,
                                       uint32_t &sv_item, uint64_t *out, uint32_t &ocount)
{
    const uint32_t c = (uint32_t)__builtin_popcount(msk);
    if (!__ballot(c != 0))
        return;
    if (lane == 0)
        *qcnt = qlen;
    __builtin_amdgcn_wave_barrier();
    uint32_t pos = 0;
    if (c)
        pos = atomicAdd(qcnt, c);
    __builtin_amdgcn_wave_barrier();
    const uint32_t tot = __builtin_amdgcn_readfirstlane(*qcnt);
    if (tot <= (uint32_t)kQueueCap) {
        while (msk) {
            const uint32_t bit = (uint32_t)__builtin_ctz(msk);
            queue[pos++] = ent0 + (bit << kWordBits);
            msk &= msk - 1u;
        }
        __builtin_amdgcn_wave_barrier();
        sv_item += tot - qlen;
        qlen = tot;
        return;
    }
    // more survivors than the queue holds (nothing was written): one half at
    // a time, each appended to a queue drained below 64 entries, so that
    // at most 63 + 64 * 16 = kQueueCap entries are held
    for (uint32_t h = 0; h < 2; ++h) {
        while (qlen >= 64)
            drain<METRIC, K>(a, it, queue, qlen, 64, lane, out, ocount);
        uint32_t m = h ? (msk >> kChunk) : (msk & 0xFFFFu);
        const uint32_t ch = (uint32_t)__builtin_popcount(m);
        if (!__ballot(ch != 0))
            continue;
        if (lane == 0)
            *qcnt = qlen;
        __builtin_amdgcn_wave_barrier();
        uint32_t p = 0;
        if (ch)
            p = atomicAdd(qcnt, ch);
        const uint32_t e1 = ent0 + ((h * kChunk) << kWordBits);
        while (m) {
            const uint32_t bit = (uint32_t)__builtin_ctz(m);
            queue[p++] = e1 + (bit << kWordBits);
            m &= m - 1u;
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t nlen = __builtin_amdgcn_readfirstlane(*qcnt);
        sv_item += nlen - qlen;
        qlen = nlen;
    }
}

// ------------------------------------------------------- matrix filter
// F_D = popc(q ^ w) of W-bit keys (W = 16 or 32) as an 8-bit integer
// contraction on the matrix cores.  Key bit j is a signed byte: 1 - 2 q_j on
// the query side and 2 w_j - 1 on the word side, so a row-column product
// over the W key positions is (differing bits) - (equal bits) = 2 F_D - W.
// One instruction covers a 32 x 32 tile with exactly W contraction
// positions (W = 32: v_mfma_i32_32x32x32_i8, 16 bytes per lane; W = 16:
// v_mfma_i32_32x32x16_i8, 8 bytes per lane): lane l holds row / column
// l % 32 and the contraction bytes of half l / 32, i.e. key bits
// (W / 2)(l / 32) .. + W / 2 - 1.  The accumulator input is the inline
// constant W - 1 - 2t (t = 2k, bigrams 4k), so each output is
// 2 F_D - 2t - 1, negative iff F_D <= t (Eq. 1), with no register tile and
// no threshold position.  A pass runs two tiles; the second one takes its
// query bytes doubled (+-2) and the constant 2W - 1 - 4t, i.e. 4 F_D - 4t -
// 1, the same sign: two different inline constants, since one constant
// shared by both instructions is moved into a 16-register tile.
//
// Output layout: lane l holds column l % 32 and, in its 16 result
// registers r, rows 8 (r / 4) + 4 (l / 32) + r % 4.  Query rows are loaded
// in a permuted order so that result register r of lane half h of the
// pass's tile t (0, 1) is query 32 h + 16 t + r: row i of tile t holds query
// 32 ((i / 4) % 2) + 16 t + 4 (i / 8) + i % 4.  Shifting the sign bits of
// tile 1's registers 15 .. 0 and then tile 0's into a mask gives bit b =
// query 32 h + b, the vector path's mask layout with 64 queries per pass.
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

// Four key bits -> four bytes: byte i is byte 0 of if_set where bit i is
// set, else byte 0 of if_clear (v_perm_b32 selector 4 picks byte 0 of its
// first operand, selector 0 byte 0 of its second).
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib, uint32_t if_set, uint32_t if_clear)
{
    const uint32_t sel = __umul24(nib, 0x00810204u) & 0x04040404u;  // bit i -> byte i = 4 * bit i
    return __builtin_amdgcn_perm(if_set, if_clear, sel);
}

// Operand types of the two tile shapes.
template <int W>
struct MxOp;
template <>
struct MxOp<16> {
    using T = long;  // 8 contraction bytes per lane
};
template <>
struct MxOp<32> {
    using T = v4i_t;  // 16 contraction bytes per lane
};

// The lane's word column: key bits (W / 2) h .. + W / 2 - 1 as bytes, +1
// for a set bit and -1 for a clear one.
template <int W>
__device__ __forceinline__ typename MxOp<W>::T word_column(uint32_t w, uint32_t h)
{
    const uint32_t x = w >> ((W / 2) * h);
    if constexpr (W == 16) {
        const uint32_t lo = nibble_bytes(x & 15u, 0x01010101u, 0xFFFFFFFFu);
        const uint32_t hi = nibble_bytes((x >> 4) & 15u, 0x01010101u, 0xFFFFFFFFu);
        return (long)(((uint64_t)hi << 32) | lo);
    } else {
        v4i_t f;
        f[0] = (int)nibble_bytes(x & 15u, 0x01010101u, 0xFFFFFFFFu);
        f[1] = (int)nibble_bytes((x >> 4) & 15u, 0x01010101u, 0xFFFFFFFFu);
        f[2] = (int)nibble_bytes((x >> 8) & 15u, 0x01010101u, 0xFFFFFFFFu);
        f[3] = (int)nibble_bytes((x >> 12) & 15u, 0x01010101u, 0xFFFFFFFFu);
        return f;
    }
}

// Shift the 16 sign bits of a tile's results into m, register 15 first.
__device__ __forceinline__ void sign_bits(const v16i_t &d, uint32_t &m)
{
#pragma unroll
    for (int r = 15; r >= 0; --r)
        m = __builtin_amdgcn_alignbit(m, (uint32_t)d[r], 31);
}

// Query bytes +-1 -> +-2 (0x01 -> 0x02, 0xFF -> 0xFE), byte by byte.
__device__ __forceinline__ uint32_t twice_bytes(uint32_t x) { return (x << 1) & 0xFEFEFEFEu; }
__device__ __forceinline__ long twice_bytes(long x)
{
    return (long)((((uint64_t)x) << 1) & 0xFEFEFEFEFEFEFEFEull);
}
__device__ __forceinline__ v4i_t twice_bytes(v4i_t x)
{
    v4i_t r;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        r[i] = (int)twice_bytes((uint32_t)x[i]);
    return r;
}

// One 32 x 32 tile: query rows qa against word columns wb, accumulator C.
template <int W, int C>
__device__ __forceinline__ void mx_tile(typename MxOp<W>::T qa, typename MxOp<W>::T wb, uint32_t &m)
{
    if constexpr (W == 16)
        sign_bits(__builtin_amdgcn_mfma_i32_32x32x16_i8(qa, wb, (v16i_t)(C), 0, 0, 0), m);
    else
        sign_bits(__builtin_amdgcn_mfma_i32_32x32x32_i8(qa, wb, (v16i_t)(C), 0, 0, 0), m);
}

// ------------------------------------------------------------ schedule

// Issue priority follows the item's position in the work list, so items
// finish roughly in the order they were taken: the hardware otherwise
// favours the oldest waves, and an item held by a young wave can run for
// most of the launch and set its tail.  Over popcount-ordered blocks with
// popcount pruning the survivors gather in the items where the two sides'
// popcounts meet, most of all where the strings are short (keys with few
// set bits: up to about 190 K survivors in one 256 x 1024 item of the 2M
// mixed workload), and the end of a launch waits for those items'
// verification; there (kOrdered), items whose shorter length is at most 7
// take the highest level whatever their position and the others the three
// below it by quartile.
template <bool kOrdered>
__device__ __forceinline__ void set_priority(uint32_t item, uint32_t n_items, uint32_t shorter)
{
    const uint32_t lvl = (uint32_t)(((uint64_t)item * 4u) / n_items);  // quartile of the list
    if (kOrdered ? shorter <= 7u : lvl == 0)
        __builtin_amdgcn_s_setprio(3);
    else if (kOrdered ? lvl == 0 : lvl == 1)
        __builtin_amdgcn_s_setprio(2);
    else if (kOrdered ? lvl == 1 : lvl == 2)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// Next item of the persistent schedule.  After the static first round of
// nw items, counter s hands out items nw + kStripes * v + s; a wave starts
// on the counter of its block's stripe and moves on to the next stripe once
// one is exhausted, so a few waves do not wait behind one contended atomic
// and no stripe is left with work.  `done` (LDS) marks the stripes a wave of
// the block found exhausted, so the end of a launch costs about one failed
// atomic per stripe and block instead of one per stripe and wave.  Returns
// n_items when every stripe is exhausted.
__device__ __forceinline__ uint32_t next_item(uint32_t *counters, uint32_t nw, uint32_t n_items, uint32_t &stripe,
                                              uint32_t &tries, uint32_t lane, uint32_t *done)
{
    while (tries < (uint32_t)kStripes) {
        // a stripe another wave of this block found exhausted costs no atomic
        if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) & (1u << stripe)) {
            stripe = (stripe + 1) % kStripes;
            ++tries;
            continue;
        }
        uint32_t v = 0;
        if (lane == 0)
            v = atomicAdd(&counters[stripe * kStripeStride], 1u);
        v = __builtin_amdgcn_readfirstlane(v);
        const uint64_t cand = (uint64_t)nw + (uint64_t)kStripes * v + stripe;
        if (cand < n_items)
            return (uint32_t)cand;
        if (lane == 0)
            __hip_atomic_fetch_or(done, 1u << stripe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        stripe = (stripe + 1) % kStripes;
        ++tries;
    }
    return n_items;
}

// Eight blocks of four waves per compute unit for the vector-ALU filter
// (64 VGPRs), seven for the matrix-core filter, whose resident query tiles
// need up to 72.
template <int KIND, int METRIC, int K, bool PERSISTENT, int MX>
__global__ void __launch_bounds__(256, MX ? 7 : 8) k_match(MatchArgs args)
{
    // The pointers used inside the loops, taken as plain values: the compiler
    // would otherwise repeat their loads from the kernel-argument segment
    // inside the loops instead of keeping them (a long-latency scalar load,
    // which the next wait on an LDS result also waits for).  Per-item
    // pointers (Item) replace base pointer + offset pairs in the drain, so
    // the filter loop keeps its own values in scalar registers.
    MatchArgs a = args;
    a.q.key = opaque_ptr(a.q.key);
    a.d.key = opaque_ptr(a.d.key);
    a.q.str = opaque_ptr(a.q.str);
    a.d.str = opaque_ptr(a.d.str);
    a.q.perm = opaque_ptr(a.q.perm);
    a.d.perm = opaque_ptr(a.d.perm);
    a.q.soff = opaque_ptr(a.q.soff);
    a.d.soff = opaque_ptr(a.d.soff);
    a.wl.pairs = opaque_ptr(a.wl.pairs);
    a.wl.counters = opaque_ptr(a.wl.counters);
    using F = Filter<KIND>;
    using Key = typename F::Key;
    __shared__ __attribute__((aligned(16))) uint32_t queue_all[kWaves][kQueueCap];
    __shared__ uint64_t out_all[kWaves][kOutCap];
    __shared__ uint32_t qcount[kWaves];
    __shared__ uint32_t s_done;  // stripes found exhausted
    if (threadIdx.x == 0)
        s_done = 0;
    __syncthreads();
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    uint32_t *queue = queue_all[wave];
    uint64_t *out = out_all[wave];
    uint32_t ocount = 0;
    const cptr<Key> qkeys = as_const((const Key *)a.q.key);
    const Key *__restrict__ dkeys = (const Key *)a.d.key;
    const uint32_t neg = filter_neg<KIND, K>();
    constexpr bool kSkip = pop_skip<KIND>();
    constexpr uint32_t kGap = pop_gap<KIND, K>();
    const uint32_t n_items = *as_const(a.wl.n_items);
    const uint32_t n_pairs = *as_const(a.wl.n_pairs);
    // survivors of the current item (wave-uniform; at most qtile x slab <=
    // 2^32 - 1 since slab < 2^22), added to the totals at the end of the
    // item (band cells: (2k + 1) min(m, L) per survivor)
    uint32_t sv_item = 0;
    uint64_t survivors = 0, cells = 0;
    // pairs of popcount-ordered blocks skipped untested (wave-uniform)
    uint64_t pruned = 0;

    // first item: the global wave index (no atomics at start-up); `wave`
    // itself stays a vector value, the item is made uniform explicitly
    const uint32_t nw = gridDim.x * kWaves;
    uint32_t stripe = blockIdx.x % kStripes, tries = 0;
    uint32_t item = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wave);
    while (item < n_items) {
        Item it = decode_item(a, item, n_pairs);
        set_priority<KIND == kPop32P || KIND == kPop64P || KIND == kQgram32P>(item, n_items, min(it.m, it.L));
        if constexpr (kSkip) {
            // the whole tile is out of popcount reach: nothing to do
            if (it.qn && it.de > it.ds &&
                pop_apart(key_pop(qkeys[it.qs]), key_pop(qkeys[it.qs + it.qn - 1]),
                          key_pop(lane_key(dkeys[it.ds], 0)), key_pop(lane_key(dkeys[it.de - 1], 0)), kGap)) {
                pruned += (uint64_t)it.qn * (it.de - it.ds);
                it.de = it.ds;
            }
        }
        uint32_t qlen = 0;
        // popcount-ordered blocks: lane c holds the key popcount range of the
        // item's query chunk c (32 queries; lo | hi << 8), read per pass with
        // one v_readlane instead of two dependent scalar loads
        uint32_t qrange = 0;
        if constexpr (kSkip) {
            if (lane < (it.qn + 31u) / 32u)
                qrange = key_pop(((const Key *)a.q.key)[it.qs + 32u * lane]) |
                         (key_pop(((const Key *)a.q.key)[it.qs + min(32u * lane + 31u, it.qn - 1u)]) << 8);
        }
        if constexpr (MX != 0) {
            // matrix cores, query-stationary: the two tiles of a group of 64
            // queries stay in registers while the slab's words stream
            // through, 32 per pass (lane: word e0 + lane % 32, queries
            // 32 (lane / 32) + b of the group)
            using Op = typename MxOp<MX>::T;
            constexpr int kT = (KIND == kQgram32 || KIND == kQgram32P) ? 4 * K : 2 * K;  // F_D threshold
            constexpr int kC1 = MX - 1 - 2 * kT, kC0 = 2 * MX - 1 - 4 * kT;
            const uint32_t h = lane >> 5, col = lane & 31u;
            const uint32_t qrow = 32u * ((col >> 2) & 1u) + 4u * (col >> 3) + (col & 3u);
            for (uint32_t j0 = 0; j0 < it.qn; j0 += 64) {
                // rows qs + j0 + 63 at most: the expanded rows carry 64 padding rows
                const uint8_t *qb = a.qexp + (size_t)(it.qs + j0 + qrow) * MX + (MX / 2) * h;
                const Op q0 = twice_bytes(*(const Op *)qb);
                const Op q1 = *(const Op *)(qb + 16u * MX);
                const uint32_t nqc = min(64u, it.qn - j0);
                const uint32_t nv = nqc > 32u * h ? min(32u, nqc - 32u * h) : 0u;
                const uint32_t qm = nv >= 32u ? ~0u : (1u << nv) - 1u;
                uint32_t plo = 0, phi = 0;  // the group's query popcount range
                if constexpr (kSkip) {
                    plo = (uint32_t)__builtin_amdgcn_readlane((int)qrange, (int)(j0 >> 5)) & 0xFFu;
                    phi = (uint32_t)__builtin_amdgcn_readlane((int)qrange, (int)((j0 + nqc - 1u) >> 5)) >> 8;
                }
                uint32_t w_next = (it.ds + col < it.de) ? dkeys[it.ds + col] : 0u;
                for (uint32_t e0 = it.ds; e0 < it.de; e0 += 32) {
                    if constexpr (kSkip) {
                        // the slab's words ascend in popcount: a group above
                        // the queries' reach ends the slab for this group
                        const uint32_t last = min(e0 + 31u, it.de - 1u) - e0;
                        const uint32_t glo = key_pop(lane_key(w_next, 0)), ghi = key_pop(lane_key(w_next, last));
                        if (glo > phi + kGap) {
                            pruned += (uint64_t)nqc * (it.de - e0);
                            break;
                        }
                        if (plo > ghi + kGap) {
                            pruned += nqc * (last + 1u);
                            w_next = (e0 + 32 + col < it.de) ? dkeys[e0 + 32 + col] : 0u;
                            continue;
                        }
                    }
                    const Op wb = word_column<MX>(w_next, h);
                    w_next = (e0 + 32 + col < it.de) ? dkeys[e0 + 32 + col] : 0u;
                    uint32_t m = 0;
                    mx_tile<MX, kC1>(q1, wb, m);
                    mx_tile<MX, kC0>(q0, wb, m);
                    if (nqc < 64u || e0 + 32 > it.de)
                        m = (e0 + col < it.de) ? m & qm : 0u;
                    append<METRIC, K>(a, it, queue, &qcount[wave], qlen, m,
                                      ((j0 + 32u * h) << kWordBits) | (e0 + col - it.ds), lane, sv_item, out, ocount);
                    while (qlen >= 64)
                        drain<METRIC, K>(a, it, queue, qlen, 64, lane, out, ocount);
                }
            }
        } else {
            // two words per lane: words e0 + lane and e0 + 64 + lane
            Key wa_next = (it.ds + lane < it.de) ? dkeys[it.ds + lane] : Key(0);
            Key wb_next = (it.ds + 64 + lane < it.de) ? dkeys[it.ds + 64 + lane] : Key(0);
            for (uint32_t e0 = it.ds; e0 < it.de; e0 += 128) {
                const Key wa = wa_next, wb = wb_next;
                wa_next = (e0 + 128 + lane < it.de) ? dkeys[e0 + 128 + lane] : Key(0);
                wb_next = (e0 + 192 + lane < it.de) ? dkeys[e0 + 192 + lane] : Key(0);
                uint32_t glo = 0, ghi = 0;
                if constexpr (kSkip) {
                    // popcount range of this group of 128 words (ascending)
                    const uint32_t last = min(e0 + 127u, it.de - 1u) - e0;
                    glo = key_pop(lane_key(wa, 0));
                    ghi = key_pop(last >= 64u ? lane_key(wb, last - 64u) : lane_key(wa, last));
                }
                uint32_t sa = 0, sb = 0;
                if constexpr (side_values<KIND>()) {
                    sa = F::side_w(wa, neg);
                    sb = F::side_w(wb, neg);
                }
                for (uint32_t j0 = 0; j0 < it.qn; j0 += 2 * kChunk) {
                    const uint32_t nqc = min(2u * kChunk, it.qn - j0);
                    const cptr<Key> qk = qkeys + it.qs + j0;  // key arrays carry 64 padding entries
                    if constexpr (kSkip) {
                        const uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)qrange, (int)(j0 >> 5));
                        if (pop_apart(r & 0xFFu, r >> 8, glo, ghi, kGap)) {
                            // the item's queries ascend in popcount: a chunk
                            // above the words' reach ends the item's chunks
                            // for this word group
                            if ((r & 0xFFu) > ghi + kGap) {
                                pruned += (it.qn - j0) * min(128u, it.de - e0);
                                break;
                            }
                            pruned += nqc * min(128u, it.de - e0);
                            continue;
                        }
                    }
                    uint32_t ma = 0, mb = 0;
                    if (nqc > (uint32_t)kChunk) {
#pragma unroll
                        for (int t = 2 * kChunk - 1; t >= kChunk; --t)
                            filter_step<KIND>(qk[t], wa, wb, sa, sb, neg, ma, mb);
                    }
#pragma unroll
                    for (int t = kChunk - 1; t >= 0; --t)
                        filter_step<KIND>(qk[t], wa, wb, sa, sb, neg, ma, mb);
                    // bit t <-> query j0 + t; drop the padding queries
                    // and the lanes past the slab (only on the item's ragged edges)
                    if (nqc < 2u * kChunk || e0 + 128 > it.de) {
                        const uint32_t qm = nqc < 32u ? (1u << nqc) - 1u : ~0u;
                        ma = (e0 + lane < it.de) ? ma & qm : 0u;
                        mb = (e0 + 64 + lane < it.de) ? mb & qm : 0u;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < 2; ++u)
                        append<METRIC, K>(a, it, queue, &qcount[wave], qlen, u ? mb : ma,
                                          (j0 << kWordBits) | (e0 + 64 * u + lane - it.ds), lane, sv_item, out,
                                          ocount);
                    while (qlen >= 64)
                        drain<METRIC, K>(a, it, queue, qlen, 64, lane, out, ocount);
                }
            }
        }
        if (qlen)
            drain<METRIC, K>(a, it, queue, qlen, qlen, lane, out, ocount);
        survivors += sv_item;
        cells += (uint64_t)((2 * K + 1) * min(it.m, it.L)) * sv_item;
        sv_item = 0;
        if (!PERSISTENT)
            break;
        item = next_item(a.wl.counters, nw, n_items, stripe, tries, lane, &s_done);
    }
    __builtin_amdgcn_s_setprio(0);
    // Block epilogue: one atomic per counter and block (the waves' last
    // atomics would otherwise all land in the launch's tail, on three
    // addresses, and slow the items still running).  The queues are empty
    // now and hold the per-wave sums.
    __syncthreads();
    uint64_t *red = (uint64_t *)&queue_all[0][0];
    if (lane == 0) {
        red[3 * wave] = survivors;
        red[3 * wave + 1] = cells;
        red[3 * wave + 2] = ocount;
        if constexpr (kSkip)
            red[3 * kWaves + 1 + wave] = pruned;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t sv = 0, ce = 0, o = 0, pr = 0, cnt[kWaves];
        for (int w = 0; w < kWaves; ++w) {
            sv += red[3 * w];
            ce += red[3 * w + 1];
            cnt[w] = red[3 * w + 2];
            if constexpr (kSkip)
                pr += red[3 * kWaves + 1 + w];
        }
        for (int w = 0; w < kWaves; ++w) {
            red[3 * w + 2] = o;  // exclusive prefix: the wave's first output slot
            o += cnt[w];
        }
        const cptr<MatchArgs> A = kargs();
        unsigned long long base = 0;
        if (o)
            base = atomicAdd((unsigned long long *)A->ctr.n_out, (unsigned long long)o);
        if (sv)
            atomicAdd((unsigned long long *)A->ctr.survivors, (unsigned long long)sv);
        if (ce)
            atomicAdd((unsigned long long *)A->ctr.verify_cells, (unsigned long long)ce);
        if (pr)
            atomicAdd((unsigned long long *)A->ctr.pruned, (unsigned long long)pr);
        red[3 * kWaves] = base;
    }
    __syncthreads();
    const uint64_t base = red[3 * kWaves] + red[3 * wave + 2];
    for (uint32_t i = lane; i < ocount; i += 64) {
        if (base + i < kargs()->out_cap)
            kargs()->out_keys[base + i] = out[i];
    }
}

// --------------------------------------------------------- work list

// Split of one compatible bucket pair (nq queries, nd words) into a
// full-size part (whole slabs, about (100 - tail_pct)% of the words) and a
// tail part of smaller tiles.
struct PairSplit {
    uint32_t nd_full, items_full, items_tail;
};

__host__ __device__ __forceinline__ uint32_t tail_qtile(uint32_t qtile) { return max(16u, (qtile / 2) & ~15u); }
__host__ __device__ __forceinline__ uint32_t tail_slab(uint32_t slab) { return max(64u, (slab / 4) & ~63u); }

__host__ __device__ __forceinline__ PairSplit split_pair(uint32_t nq, uint32_t nd, uint32_t qtile, uint32_t slab,
                                                        uint32_t tail_pct)
{
    PairSplit r;
    if (tail_pct == 0) {
        r.nd_full = nd;
    } else {
        const uint32_t keep = nd - (uint32_t)((uint64_t)nd * tail_pct / 100);
        r.nd_full = keep / slab * slab;
    }
    const uint32_t nd_tail = nd - r.nd_full;
    r.items_full = r.nd_full ? ((nq + qtile - 1) / qtile) * ((r.nd_full + slab - 1) / slab) : 0;
    const uint32_t qt = tail_qtile(qtile), sl = tail_slab(slab);
    r.items_tail = nd_tail ? ((nq + qt - 1) / qt) * ((nd_tail + sl - 1) / sl) : 0;
    return r;
}

__host__ __device__ __forceinline__ PairRec make_rec(uint32_t item_base, uint32_t qbase, uint32_t nq, uint32_t dbase,
                                                    uint32_t nd, uint32_t qtile, uint32_t slab, uint32_t m, uint32_t L)
{
    PairRec P;
    P.item_base = item_base;
    P.qbase = qbase;
    P.nq = nq;
    P.dbase = dbase;
    P.nd = nd;
    P.tiles_d = (nd + slab - 1) / slab;
    P.qlen = m;
    P.dlen = L;
    P.qtile = qtile;
    P.slab = slab;
    return P;
}

// One block: thread t owns query length m (descending or ascending order)
// and its up to 2k+1 compatible word lengths.  Four scans over the threads
// place the full records (and their items) before every tail record.
__global__ void __launch_bounds__(256) k_worklist(const uint32_t *qoff, const uint32_t *doff, int metric, uint32_t k,
                                                  uint32_t qtile, uint32_t slab, uint32_t order, uint32_t tail_pct,
                                                  WorkList wl)
{
    __shared__ uint32_t s_cnt[4][256];  // full records, full items, tail records, tail items
    __shared__ unsigned long long s_exam[256];
    const uint32_t t = threadIdx.x;
    const int m = order == 0 ? 255 - (int)t : (int)t;
    const uint32_t nq = qoff[m + 1] - qoff[m];
    const int r = metric == 0 ? 0 : (int)k;
    uint32_t c[4] = {0, 0, 0, 0};
    unsigned long long ex = 0;
    if (nq) {
        for (int L = m - r; L <= m + r; ++L) {
            if (L < 0 || L > 255)
                continue;
            const uint32_t nd = doff[L + 1] - doff[L];
            if (!nd)
                continue;
            const PairSplit sp = split_pair(nq, nd, qtile, slab, tail_pct);
            c[0] += sp.items_full ? 1 : 0;
            c[1] += sp.items_full;
            c[2] += sp.items_tail ? 1 : 0;
            c[3] += sp.items_tail;
            ex += (unsigned long long)nq * nd;
        }
    }
    for (int v = 0; v < 4; ++v)
        s_cnt[v][t] = c[v];
    s_exam[t] = ex;
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        uint32_t add[4];
        for (int v = 0; v < 4; ++v)
            add[v] = t >= o ? s_cnt[v][t - o] : 0;
        const unsigned long long e = t >= o ? s_exam[t - o] : 0;
        __syncthreads();
        for (int v = 0; v < 4; ++v)
            s_cnt[v][t] += add[v];
        s_exam[t] += e;
        __syncthreads();
    }
    const uint32_t full_pairs = s_cnt[0][255], full_items = s_cnt[1][255];
    uint32_t pf = s_cnt[0][t] - c[0], ifull = s_cnt[1][t] - c[1];
    uint32_t pt = full_pairs + s_cnt[2][t] - c[2], itail = full_items + s_cnt[3][t] - c[3];
    if (nq) {
        const uint32_t qt2 = tail_qtile(qtile), sl2 = tail_slab(slab);
        for (int L = m - r; L <= m + r; ++L) {
            if (L < 0 || L > 255)
                continue;
            const uint32_t nd = doff[L + 1] - doff[L];
            if (!nd)
                continue;
            const PairSplit sp = split_pair(nq, nd, qtile, slab, tail_pct);
            if (sp.items_full) {
                wl.pairs[pf++] = make_rec(ifull, qoff[m], nq, doff[L], sp.nd_full, qtile, slab, (uint32_t)m, (uint32_t)L);
                ifull += sp.items_full;
            }
            if (sp.items_tail) {
                wl.pairs[pt++] = make_rec(itail, qoff[m], nq, doff[L] + sp.nd_full, nd - sp.nd_full, qt2, sl2,
                                          (uint32_t)m, (uint32_t)L);
                itail += sp.items_tail;
            }
        }
    }
    if (t == 255) {
        *wl.n_pairs = full_pairs + s_cnt[2][255];
        *wl.n_items = full_items + s_cnt[3][255];
        *wl.examined = s_exam[255];
    }
}

template <int METRIC, int K>
__global__ void k_verify_pairs(StrSetView q, const uint32_t *qinv, StrSetView d, const uint32_t *dinv,
                               const uint32_t *pairs, uint64_t n, uint32_t *dist)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t qi = qinv[pairs[2 * i]], wi = dinv[pairs[2 * i + 1]];
    dist[i] = verify<METRIC, K>(q.str + q.soff[qi], q.len[qi], d.str + d.soff[wi], d.len[wi]);
}

template <int KIND, int METRIC, int K, int MX = 0>
hipError_t launch_kmk(const MatchArgs &a, bool persistent, uint32_t pblocks, uint32_t host_items, hipStream_t s)
{
    if (persistent) {
        hipLaunchKernelGGL((k_match<KIND, METRIC, K, true, MX>), dim3(pblocks), dim3(256), 0, s, a);
    } else {
        if (host_items == 0)
            return hipSuccess;
        hipLaunchKernelGGL((k_match<KIND, METRIC, K, false, MX>), dim3((host_items + kWaves - 1) / kWaves), dim3(256),
                           0, s, a);
    }
    return hipGetLastError();
}

template <int KIND, int MX = 0>
hipError_t launch_kind(const MatchArgs &a, int metric, uint32_t k, bool persistent, uint32_t pblocks,
                       uint32_t host_items, hipStream_t s)
{
    if (metric == 0) {
        if (k == 1)
            return launch_kmk<KIND, 0, 1, MX>(a, persistent, pblocks, host_items, s);
        if (k == 2)
            return launch_kmk<KIND, 0, 2, MX>(a, persistent, pblocks, host_items, s);
        return launch_kmk<KIND, 0, 3, MX>(a, persistent, pblocks, host_items, s);
    }
    if (k == 1)
        return launch_kmk<KIND, 1, 1, MX>(a, persistent, pblocks, host_items, s);
    if (k == 2)
        return launch_kmk<KIND, 1, 2, MX>(a, persistent, pblocks, host_items, s);
    return launch_kmk<KIND, 1, 3, MX>(a, persistent, pblocks, host_items, s);
}

// Query rows of the matrix filter: key bit j as byte j of the row, +1 for a
// clear bit (0x01) and -1 for a set bit (0xFF); width bytes per query.
__global__ void k_expand_keys(const uint32_t *keys, uint32_t n, uint32_t width, uint8_t *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t key = keys[i];
    uint4 v;
    v.x = nibble_bytes(key & 15u, 0xFFFFFFFFu, 0x01010101u);
    v.y = nibble_bytes((key >> 4) & 15u, 0xFFFFFFFFu, 0x01010101u);
    v.z = nibble_bytes((key >> 8) & 15u, 0xFFFFFFFFu, 0x01010101u);
    v.w = nibble_bytes((key >> 12) & 15u, 0xFFFFFFFFu, 0x01010101u);
    uint4 *row = (uint4 *)(out + (size_t)i * width);
    row[0] = v;
    if (width == 32) {
        v.x = nibble_bytes((key >> 16) & 15u, 0xFFFFFFFFu, 0x01010101u);
        v.y = nibble_bytes((key >> 20) & 15u, 0xFFFFFFFFu, 0x01010101u);
        v.z = nibble_bytes((key >> 24) & 15u, 0xFFFFFFFFu, 0x01010101u);
        v.w = nibble_bytes((key >> 28) & 15u, 0xFFFFFFFFu, 0x01010101u);
        row[1] = v;
    }
}

}  // namespace

uint32_t host_worklist(const uint32_t *qoff, const uint32_t *doff, int metric, uint32_t k, uint32_t qtile,
                       uint32_t slab, uint32_t order, PairRec *pairs, uint32_t *n_pairs, uint64_t *examined)
{
    const int r = metric == 0 ? 0 : (int)k;
    uint32_t np = 0, items = 0;
    uint64_t ex = 0;
    for (int t = 0; t < 256; ++t) {
        const int m = order == 0 ? 255 - t : t;
        const uint32_t nq = qoff[m + 1] - qoff[m];
        if (!nq)
            continue;
        for (int L = m - r; L <= m + r; ++L) {
            if (L < 0 || L > 255)
                continue;
            const uint32_t nd = doff[L + 1] - doff[L];
            if (!nd)
                continue;
            pairs[np] = make_rec(items, qoff[m], nq, doff[L], nd, qtile, slab, (uint32_t)m, (uint32_t)L);
            items += ((nq + qtile - 1) / qtile) * pairs[np].tiles_d;
            ++np;
            ex += (uint64_t)nq * nd;
        }
    }
    *n_pairs = np;
    *examined = ex;
    return items;
}

void launch_worklist(const uint32_t *qoff, const uint32_t *doff, int metric, uint32_t k, uint32_t qtile,
                     uint32_t slab, uint32_t order, uint32_t tail_pct, WorkList wl, hipStream_t s)
{
    hipLaunchKernelGGL(k_worklist, dim3(1), dim3(256), 0, s, qoff, doff, metric, k, qtile, slab, order, tail_pct, wl);
}

void launch_expand_keys(const uint32_t *keys, uint32_t n, int width, uint8_t *out, hipStream_t s)
{
    if (n)
        hipLaunchKernelGGL(k_expand_keys, dim3((n + 255) / 256), dim3(256), 0, s, keys, n, (uint32_t)width, out);
}

hipError_t launch_match(const MatchArgs &a, int key_kind, int key_width, int metric, uint32_t k, bool persistent,
                        uint32_t persistent_blocks, uint32_t host_items, hipStream_t s)
{
    if (key_width) {
        if (key_width != 16 && key_width != 32)
            return hipErrorInvalidValue;
        const bool w16 = key_width == 16;
        switch (key_kind) {
        case kPop32:
            return w16 ? launch_kind<kPop32, 16>(a, metric, k, persistent, persistent_blocks, host_items, s)
                       : launch_kind<kPop32, 32>(a, metric, k, persistent, persistent_blocks, host_items, s);
        case kQgram32:
            return w16 ? launch_kind<kQgram32, 16>(a, metric, k, persistent, persistent_blocks, host_items, s)
                       : launch_kind<kQgram32, 32>(a, metric, k, persistent, persistent_blocks, host_items, s);
        case kPop32P:
            return w16 ? launch_kind<kPop32P, 16>(a, metric, k, persistent, persistent_blocks, host_items, s)
                       : launch_kind<kPop32P, 32>(a, metric, k, persistent, persistent_blocks, host_items, s);
        case kQgram32P:
            return w16 ? launch_kind<kQgram32P, 16>(a, metric, k, persistent, persistent_blocks, host_items, s)
                       : launch_kind<kQgram32P, 32>(a, metric, k, persistent, persistent_blocks, host_items, s);
        default:
            return hipErrorInvalidValue;
        }
    }
    switch (key_kind) {
    case kPop32:
        return launch_kind<kPop32>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kPop64:
        return launch_kind<kPop64>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kPos16:
        if (metric != 0)
            return hipErrorInvalidValue;
        return k == 1   ? launch_kmk<kPos16, 0, 1>(a, persistent, persistent_blocks, host_items, s)
               : k == 2 ? launch_kmk<kPos16, 0, 2>(a, persistent, persistent_blocks, host_items, s)
                        : launch_kmk<kPos16, 0, 3>(a, persistent, persistent_blocks, host_items, s);
    case kPos32:
        if (metric != 0)
            return hipErrorInvalidValue;
        return k == 1   ? launch_kmk<kPos32, 0, 1>(a, persistent, persistent_blocks, host_items, s)
               : k == 2 ? launch_kmk<kPos32, 0, 2>(a, persistent, persistent_blocks, host_items, s)
                        : launch_kmk<kPos32, 0, 3>(a, persistent, persistent_blocks, host_items, s);
    case kTherm32:
        return launch_kind<kTherm32>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kAsym32:
        return launch_kind<kAsym32>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kAsym64:
        return launch_kind<kAsym64>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kQgram32:
        return launch_kind<kQgram32>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kCombo64:
        return launch_kind<kCombo64>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kPop32P:
        return launch_kind<kPop32P>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kPop64P:
        return launch_kind<kPop64P>(a, metric, k, persistent, persistent_blocks, host_items, s);
    case kQgram32P:
        return launch_kind<kQgram32P>(a, metric, k, persistent, persistent_blocks, host_items, s);
    default:
        return launch_kind<kAll>(a, metric, k, persistent, persistent_blocks, host_items, s);
    }
}

hipError_t launch_verify_pairs(StrSetView q, const uint32_t *qinv, StrSetView d, const uint32_t *dinv,
                               const uint32_t *pairs, uint64_t n, int metric, uint32_t k, uint32_t *dist,
                               hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const dim3 g((uint32_t)((n + 255) / 256)), b(256);
#define FPM_VERIFY_PAIRS(M, K) hipLaunchKernelGGL((k_verify_pairs<M, K>), g, b, 0, s, q, qinv, d, dinv, pairs, n, dist)
    if (metric == 0) {
        if (k == 1)
            FPM_VERIFY_PAIRS(0, 1);
        else if (k == 2)
            FPM_VERIFY_PAIRS(0, 2);
        else
            FPM_VERIFY_PAIRS(0, 3);
    } else {
        if (k == 1)
            FPM_VERIFY_PAIRS(1, 1);
        else if (k == 2)
            FPM_VERIFY_PAIRS(1, 2);
        else
            FPM_VERIFY_PAIRS(1, 3);
    }
#undef FPM_VERIFY_PAIRS
    return hipGetLastError();
}

}  // namespace fpm
