// fpm_internal.hpp -- internal declarations shared by the HIP sources of
// libfpm (device-side data layout, kernel launch wrappers).
//
// Device layout of a string set (dictionary or query batch), all in HBM:
//   * strings are stably sorted by length; strings of length L occupy the
//     sorted positions [off[L], off[L+1]);
//   * each string is copied into a zero-padded slot of sw(L) dwords: 1 for
//     L <= 4, 2 for L <= 8, else 4 * ceil(L / 16), so that a slot is read
//     with one dword, one dwordx2 or dwordx4 loads; the slots of one length
//     form one dense block whose base is 16-byte aligned;
//     soff[p] is the dword offset of sorted string p, len[p] its length and
//     perm[p] its position in the caller's list;
//   * key[p] is the filter key of string p (see fpm_match.hip): the
//     fingerprint itself, or for the count variant its thermometer
//     expansion, so that one XOR and one popcount give F_D.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpm {

constexpr int kMaxLen = 255;
constexpr int kBuckets = 256;        // lengths 0..255
constexpr int kMaxK = 3;                // largest supported k (match keys hold the distance in 2 bits)
constexpr int kMaxPairs = 2 * 256 * (2 * kMaxK + 1);  // (query length, word length) pairs, |dL| <= k, full + tail part
constexpr int kRadixShift = 8;
constexpr int kRadixBlocks = 1 << kRadixShift;  // blocks of one stable radix pass (16 waves each)
constexpr int kSortBits = 10;                   // digit width of the match-list sort (lengths use 8)
// uint32 scratch of a pass: the digit table [bins][kRadixBlocks], then the
// bins' totals
constexpr size_t kRadixScratch = ((size_t)kRadixBlocks << kSortBits) + (1u << kSortBits);

__host__ __device__ inline uint32_t slot_dwords(uint32_t len)
{
    return len <= 4 ? 1u : len <= 8 ? 2u : 4u * ((len + 15u) >> 4);
}

// Filter-key families.  Pop32: F_D = popc(kq ^ kw) on 32-bit keys (occ,
// occ-halved, 16-bit count thermometer); Pop64: the same on 64-bit keys
// (32-bit count thermometer); Pos16 / Pos32: position fingerprints; All: no
// filter (brute force, every length-compatible pair is verified).
// The asymmetric bound max(popc(q & ~w), popc(w & ~q)) <= k (an extension
// of Eq. 1, sound wherever F_D is) uses:
//   Therm32: a 16-bit key with the thermometer code of its own popcount in
//            bits 16..31, so popc(kq ^ kw) = F_D + |pq - pw| = twice the
//            larger excess and the Pop32 test applies unchanged;
//   Asym32 / Asym64: the Pop32 / Pop64 keys, tested as
//            popc(~(q & w)) + max(pq, pw) against the key width + k + 1.
// Qgram32: bigram fingerprints, F_D = popc(kq ^ kw) rejected above 4k (one
// edit replaces at most two bigrams).  Combo64: combined occurrence + count
// fingerprints, the occurrence half in the low word and the counters'
// thermometer expansion in the high word; a pair survives when both words'
// XOR popcounts are <= 2k.
// Pop32P / Pop64P / Qgram32P: the Pop32 / Pop64 / Qgram32 keys and test over
// a dictionary and a query batch whose length blocks are ordered by key
// popcount: since F_D = popc(kq ^ kw) >= |pq - pw|, a group of pairs whose
// popcount ranges lie more than the threshold apart cannot survive and is
// skipped untested (kernel variants only; the keys are the base kind's).
enum KeyKind : int {
    kPop32 = 0,
    kPop64 = 1,
    kPos16 = 2,
    kPos32 = 3,
    kAll = 4,
    kTherm32 = 5,
    kAsym32 = 6,
    kAsym64 = 7,
    kQgram32 = 8,
    kCombo64 = 9,
    kPop32P = 10,
    kPop64P = 11,
    kQgram32P = 12
};

__host__ __device__ inline bool key_is_64(int kind)
{
    return kind == kPop64 || kind == kAsym64 || kind == kCombo64 || kind == kPop64P;
}

// The popcount-ordered kernel variant of a key kind (-1: none).
__host__ __device__ inline int pop_pruned_kind(int kind)
{
    return kind == kPop32 ? kPop32P : kind == kPop64 ? kPop64P : kind == kQgram32 ? kQgram32P : -1;
}

struct StrSetView {
    const uint32_t *perm;  // sorted -> caller index
    const uint8_t *len;    // sorted -> length
    const uint32_t *soff;  // sorted -> dword offset of the padded string
    const uint32_t *str;   // padded strings
    const uint32_t *off;   // [257] bucket offsets
    const void *key;       // filter keys (uint32 or uint64), sorted order
};

// One (query length, word length) pair of buckets and its work items.
struct PairRec {
    uint32_t item_base;  // first work item of this pair
    uint32_t qbase, nq;  // sorted query range
    uint32_t dbase, nd;  // sorted dictionary range
    uint32_t tiles_d;    // dictionary slabs per query tile
    uint32_t qlen, dlen;
    uint32_t qtile, slab;  // tile of this record's items
};

// The persistent schedule hands out work items through kStripes counters,
// kStripeStride words apart (one per cache line): counter s serves items
// nw + kStripes * v + s after the static first round of nw items.
constexpr int kStripes = 8;
constexpr int kStripeStride = 64;

struct WorkList {
    PairRec *pairs;       // [kMaxPairs]
    uint32_t *n_pairs;    // device scalar
    uint32_t *n_items;    // device scalar
    uint32_t *counters;   // [kStripes * kStripeStride], zero before a persistent launch
    uint64_t *examined;   // device scalar: length-compatible pairs
};

struct MatchCounters {
    uint64_t *n_out;        // matches found (may exceed capacity)
    uint64_t *survivors;    // pairs verified
    uint64_t *verify_cells; // sum (2k+1) * min(m, n)
    uint64_t *pruned;       // examined pairs skipped by popcount order (never tested)
};

// Destination of the last pass of the match-list sort (out == nullptr: none).
struct Unpack {
    uint32_t *out = nullptr;
    uint32_t wbits = 0;
    int pairs_only = 0;
};

struct MatchArgs {
    StrSetView q, d;
    WorkList wl;
    MatchCounters ctr;
    uint64_t *out_keys;   // packed (query, word, dist) keys
    uint64_t out_cap;
    uint32_t wbits;       // bits of a word index in the packed key
    uint32_t survivors_only;  // 1: report every survivor with dist 0, no verification
    // matrix-core filter: the query keys as signed bytes (launch_expand_keys),
    // key_width bytes per sorted query, 64 padding rows
    const uint8_t *qexp;
};

// ----------------------------------------------------------------- build
// Lengths of a CSR list, clamped to kMaxLen; err gets bit 1 for a long
// string, bit 2 for decreasing offsets.  Reads offsets[0..n].
void launch_lengths(const uint64_t *offsets, uint32_t n, uint32_t *len_out, uint32_t *err, hipStream_t s);

// Byte histogram of bytes[offsets[0] .. offsets[n]) into hist[256].
void launch_byte_histogram(const uint8_t *bytes, const uint64_t *offsets, uint32_t n, unsigned long long *hist,
                           hipStream_t s);
// Symbol map from a histogram (common / rare / mixed), map_out[256].
void launch_select_symbols(const unsigned long long *hist, int nfields, int symset, uint8_t *map_out, hipStream_t s);

// Reorder a laid-out set (block tables off / bdw, padded strings, sorted ->
// caller perm, keys of key_kind) inside each length block by key popcount,
// stably, into str_out / perm_out / keys_out (slot offsets and lengths are
// per position and stay valid).  One launch, one block per length.
void launch_pop_order(const uint32_t *off, const uint32_t *bdw, const uint32_t *str, const uint32_t *perm,
                      const void *keys, int key_kind, uint32_t *str_out, uint32_t *perm_out, void *keys_out,
                      hipStream_t s);

// Stable sort of indices 0..n-1 by length (a single 8-bit radix pass).
// Writes perm (sorted -> caller index), off[257] bucket offsets and
// bdw[257] dword offsets of the padded blocks.  scratch: kRadixScratch
// uint32.
void launch_length_sort(const uint32_t *len, uint32_t n, uint32_t *perm, uint32_t *off, uint32_t *bdw,
                        uint32_t *scratch, hipStream_t s);

// Padded copy of the strings in sorted order; writes slen, soff, str.
// Reads bytes below min(nbytes_limit, offsets[n]); slots past str_cap dwords
// are refused (err bit 4).
void launch_layout(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit, const uint32_t *perm,
                   const uint32_t *len, const uint32_t *off, const uint32_t *bdw, uint32_t n, uint8_t *slen,
                   uint32_t *soff, uint32_t *str, uint64_t str_cap, uint32_t *err, hipStream_t s);

// launch_layout and the fingerprints (Section 3.2) of the strings in one
// pass: fp_orig[perm[p]] (optional) and the filter keys (required).
void launch_layout_fp(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit, const uint32_t *perm,
                      const uint32_t *len, const uint32_t *off, const uint32_t *bdw, uint32_t n, uint8_t *slen,
                      uint32_t *soff, uint32_t *str, uint64_t str_cap, uint32_t *err, const uint8_t *map, int variant,
                      int bits, uint32_t *fp_orig, void *keys, int key_kind, hipStream_t s);

// Fingerprints (Section 3.2) of the sorted padded strings: fp_sorted[p],
// fp_orig[perm[p]] (optional) and the filter keys.
void launch_fingerprints(const uint32_t *str, const uint32_t *soff, const uint8_t *slen, const uint32_t *perm,
                         uint32_t n, const uint8_t *map, int variant, int bits, uint32_t *fp_sorted,
                         uint32_t *fp_orig, void *keys, int key_kind, hipStream_t s);

// Zero n uint32 words with a kernel (safe inside graph capture).
void launch_zero(void *p, size_t n_u32, hipStream_t s);

// ----------------------------------------------------------------- match
// Device work list: for every compatible bucket pair a full-size record
// (whole slabs covering about (100 - tail_pct)% of its words) and a tail
// record of (qtile / 2) x (slab / 4) tiles for the rest; all full records
// come first.  tail_pct = 0: full records only.
void launch_worklist(const uint32_t *qoff, const uint32_t *doff, int metric, uint32_t k, uint32_t qtile,
                     uint32_t slab, uint32_t order, uint32_t tail_pct, WorkList wl, hipStream_t s);
// host-side twin used by the plain schedule
uint32_t host_worklist(const uint32_t *qoff, const uint32_t *doff, int metric, uint32_t k, uint32_t qtile,
                       uint32_t slab, uint32_t order, PairRec *pairs, uint32_t *n_pairs, uint64_t *examined);

// Launch the fused filter -> LDS queue -> verify kernel.
//   persistent: grid = persistent_blocks; wave w takes item w first, then
//   items from the striped counters;
//   otherwise grid covers host_items items, one per wave.
//   key_width 16 or 32: the filter test runs on the matrix cores over keys
//   of that many bits (key kinds kPop32 and kQgram32 only; a.qexp filled
//   by launch_expand_keys); 0: on the vector ALUs.
hipError_t launch_match(const MatchArgs &a, int key_kind, int key_width, int metric, uint32_t k, bool persistent,
                        uint32_t persistent_blocks, uint32_t host_items, hipStream_t s);

// Query side of the matrix-core filter: each of the n keys becomes a row of
// width (16 or 32) signed bytes, byte j = +1 for a clear bit j, -1 for a set
// one.  The buffer holds kMxRowBytes bytes per query plus 64 padding rows.
constexpr int kMxRowBytes = 32;
void launch_expand_keys(const uint32_t *keys, uint32_t n, int width, uint8_t *out, hipStream_t s);

// Exact distances of explicit (query, word) pairs given as caller indices;
// qinv / dinv map caller index -> sorted position.
hipError_t launch_verify_pairs(StrSetView q, const uint32_t *qinv, StrSetView d, const uint32_t *dinv,
                               const uint32_t *pairs, uint64_t n, int metric, uint32_t k, uint32_t *dist,
                               hipStream_t s);

// Inverse permutation: inv[perm[p]] = p.
void launch_invert(const uint32_t *perm, uint32_t n, uint32_t *inv, hipStream_t s);

// ----------------------------------------------------------------- sort
// Stable LSD radix sort of packed match keys (count read from device,
// clamped to cap) on bits [lo_bit, hi_bit), kSortBits per pass, ping-pong
// between keys and tmp; the last pass writes each key straight to triples as
// (query, word, dist) (pairs_only: (query, word)), word = the wbits above
// the 2 dist bits.  scratch: kRadixScratch uint32.
void launch_sort_unpack(uint64_t *keys, uint64_t *tmp, const uint64_t *count, uint64_t cap, uint32_t lo_bit,
                        uint32_t hi_bit, uint32_t wbits, uint32_t *triples, int pairs_only, uint32_t *scratch,
                        hipStream_t s);

}  // namespace fpm
