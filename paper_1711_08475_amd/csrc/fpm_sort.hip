// fpm_sort.hip -- stable LSD radix sort passes used for the length bucketing
// of dictionaries and query batches (8-bit digits) and for the final
// (query, word) ordering of the match list (kSortBits-bit digits).
//
// One pass = three launches:
//   hist:    kRadixBlocks blocks each count the digits of a contiguous range;
//   scan:    one wave per digit row of the digit-major table
//            [bins][kRadixBlocks] turns it into exclusive offsets within the
//            row and writes the digit's total; the scatter adds the totals of
//            the smaller digits, so block b's first item of digit d goes to
//            sum(totals[< d]) + offs[d][b];
//   scatter: each block splits its range into kScatterWaves contiguous
//            sub-ranges, counts their digits in LDS, derives each wave's
//            starting offsets, and every wave walks its sub-range in order,
//            64 items at a time; lanes with equal digits are found with one
//            ballot per digit bit, so the rank of a lane among equal digits is the
//            popcount of its peers below it -- the pass is stable.
// The item count may live in device memory (match list), so every kernel
// splits [0, n) into kRadixBlocks ranges at run time.
#include "fpm_internal.hpp"

namespace fpm {

namespace {

__device__ __forceinline__ uint64_t range_n(const uint64_t *dcount, uint64_t hcount, uint64_t cap)
{
    if (!dcount)
        return hcount;
    uint64_t n = *dcount;
    return n < cap ? n : cap;
}

template <typename K, int BITS>
__global__ void __launch_bounds__(256) k_radix_hist(const K *keys, const uint64_t *dcount, uint64_t hcount,
                                                    uint64_t cap, uint32_t shift, uint32_t *hist)
{
    constexpr uint32_t BINS = 1u << BITS, MASK = BINS - 1u;
    __shared__ uint32_t h[BINS];
    const uint32_t b = blockIdx.x;
    for (uint32_t d = threadIdx.x; d < BINS; d += 256)
        h[d] = 0;
    __syncthreads();
    const uint64_t n = range_n(dcount, hcount, cap);
    const uint64_t lo = n * b / kRadixBlocks, hi = n * (b + 1) / kRadixBlocks;
    // eight independent loads in flight per thread before their LDS adds
    uint64_t i = lo + threadIdx.x;
    for (; i + 7 * 256 < hi; i += 8 * 256) {
        uint32_t d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            d[u] = (uint32_t)(keys[i + u * 256] >> shift) & MASK;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            atomicAdd(&h[d[u]], 1u);
    }
    for (; i < hi; i += 256)
        atomicAdd(&h[(uint32_t)(keys[i] >> shift) & MASK], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < BINS; d += 256)
        hist[d * kRadixBlocks + b] = h[d];
}

// Inclusive prefix sum over the 64 lanes of a wave (shuffles).
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= (uint32_t)off)
            v += y;
    }
    return v;
}

// Row scans of the digit-major table [BINS][kRadixBlocks]: one wave per
// digit row (kRadixBlocks / 64 entries per lane, read and written
// coalesced) turns the row into exclusive offsets within the row and writes
// the row total (the digit's count) to totals[digit].  Rows are independent,
// so the pass spreads over BINS / 16 blocks; the offsets of the rows before
// a digit are added where they are used (scatter, bucket tables).
__global__ void __launch_bounds__(1024) k_scan_rows(uint32_t *v, uint32_t *totals)
{
    constexpr int PL = kRadixBlocks / 64;  // entries per lane and row
    static_assert(kRadixBlocks % 64 == 0, "rows are split evenly over the lanes");
    const uint32_t lane = threadIdx.x & 63u, row = blockIdx.x * 16u + (threadIdx.x >> 6);
    uint32_t *r = v + (size_t)row * kRadixBlocks + lane * PL;
    uint32_t x[PL], sum = 0;
#pragma unroll
    for (int e = 0; e < PL; ++e) {
        x[e] = r[e];
        sum += x[e];
    }
    const uint32_t inc = wave_inclusive(sum, lane);
    uint32_t run = inc - sum;
#pragma unroll
    for (int e = 0; e < PL; ++e) {
        r[e] = run;
        run += x[e];
    }
    if (lane == 63)
        totals[row] = inc;
}

// Exclusive prefix over digits of the BINS row totals, into base[] (LDS), by
// a block of at least BINS threads.  wsum: one LDS word per wave.
template <int BINS>
__device__ __forceinline__ void digit_bases(const uint32_t *totals, uint32_t *base, uint32_t *wsum)
{
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t c = t < (uint32_t)BINS ? totals[t] : 0u;
    const uint32_t inc = wave_inclusive(c, lane);
    if (t < (uint32_t)BINS && lane == 63)
        wsum[w] = inc;
    __syncthreads();
    if (t < (uint32_t)BINS) {
        uint32_t ex = inc - c;
        for (uint32_t j = 0; j < w; ++j)
            ex += wsum[j];
        base[t] = ex;
    }
    __syncthreads();
}

// Packed match key (query | word | dist, dist in the low 2 bits, the word
// in the next wbits) -> (query, word, dist) triple, or (query, word) pair.
__device__ __forceinline__ void unpack_key(uint64_t k, uint64_t pos, const Unpack &u)
{
    const uint64_t wmask = (u.wbits >= 64) ? ~0ull : ((1ull << u.wbits) - 1ull);
    const uint32_t d = (uint32_t)(k & 3ull);
    const uint32_t w = (uint32_t)((k >> 2) & wmask);
    const uint32_t q = (uint32_t)(k >> (2 + u.wbits));
    if (u.pairs_only) {
        u.out[2 * pos] = q;
        u.out[2 * pos + 1] = w;
    } else {
        u.out[3 * pos] = q;
        u.out[3 * pos + 1] = w;
        u.out[3 * pos + 2] = d;
    }
}

// kScatterWaves waves per block.  vals_in == nullptr means value = item index.
// With un.out set (last pass of the match-list sort) a key is written as its
// unpacked triple at its sorted position instead.
constexpr int kScatterWaves = 16;

template <typename K, int BITS>
__global__ void __launch_bounds__(64 * kScatterWaves) k_radix_scatter(const K *keys_in, const uint32_t *vals_in,
                                                                      K *keys_out, uint32_t *vals_out,
                                                                      const uint64_t *dcount, uint64_t hcount,
                                                                      uint64_t cap, uint32_t shift,
                                                                      const uint32_t *offs, Unpack un)
{
    constexpr uint32_t BINS = 1u << BITS, MASK = BINS - 1u;
    static_assert(BINS <= 64 * kScatterWaves, "one thread per digit in the prefix step");
    __shared__ uint32_t run[kScatterWaves][BINS];
    __shared__ uint32_t base[BINS];
    __shared__ uint32_t wsum[kScatterWaves];
    const uint32_t b = blockIdx.x, lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < kScatterWaves * BINS; i += blockDim.x)
        (&run[0][0])[i] = 0;
    digit_bases<BINS>(offs + ((size_t)BINS << kRadixShift), base, wsum);
    const uint64_t n = range_n(dcount, hcount, cap);
    const uint64_t blo = n * b / kRadixBlocks, bhi = n * (b + 1) / kRadixBlocks;
    const uint64_t lo = blo + (bhi - blo) * w / kScatterWaves, hi = blo + (bhi - blo) * (w + 1) / kScatterWaves;
    // digit counts of each wave's sub-range
    for (uint64_t i = lo + lane; i < hi; i += 64)
        atomicAdd(&run[w][(uint32_t)(keys_in[i] >> shift) & MASK], 1u);
    __syncthreads();
    // exclusive prefix over the waves, starting at the block's offsets
    if (threadIdx.x < BINS) {
        const uint32_t d = threadIdx.x;
        uint32_t r = base[d] + offs[d * kRadixBlocks + b];
        for (int ww = 0; ww < kScatterWaves; ++ww) {
            const uint32_t c = run[ww][d];
            run[ww][d] = r;
            r += c;
        }
    }
    __syncthreads();
    uint32_t *running = run[w];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    K next = (lo + lane < hi) ? keys_in[lo + lane] : K(0);
    for (uint64_t base = lo; base < hi; base += 64) {
        const uint64_t i = base + lane;
        const bool active = i < hi;
        const K key = next;
        next = (i + 64 < hi) ? keys_in[i + 64] : K(0);  // prefetch the next group
        uint32_t val = 0;
        if (active)
            val = vals_in ? vals_in[i] : (uint32_t)i;
        const uint32_t digit = (uint32_t)(key >> shift) & MASK;
        uint64_t peers = __ballot(active);
#pragma unroll
        for (int bit = 0; bit < BITS; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t start = running[digit];
        __builtin_amdgcn_wave_barrier();
        if (active) {
            const uint32_t rank = (uint32_t)__popcll(peers & below);
            const uint32_t pos = start + rank;
            if (un.out)
                unpack_key((uint64_t)key, pos, un);
            else if (keys_out)
                keys_out[pos] = key;
            if (vals_out)
                vals_out[pos] = val;
            if (rank == 0)
                running[digit] = start + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Bucket tables from the scanned digit table of a length pass:
// off[L] = first sorted position of length L, bdw[L] = first dword of the
// padded block of length L.
__global__ void __launch_bounds__(256) k_bucket_tables(const uint32_t *offs, uint32_t n, uint32_t *off,
                                                       uint32_t *bdw)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t wsum[4];
    const uint32_t L = threadIdx.x;
    const uint32_t *counts = offs + ((size_t)256 << kRadixShift);  // row totals of the 8-bit length pass
    digit_bases<256>(counts, base, wsum);
    off[L] = base[L];
    if (L == 255)
        off[256] = n;
    part[L] = (counts[L] * slot_dwords(L) + 3u) & ~3u;  // 16-byte aligned blocks
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        uint32_t x = L >= o ? part[L - o] : 0;
        __syncthreads();
        part[L] += x;
        __syncthreads();
    }
    bdw[L] = L ? part[L - 1] : 0;
    if (L == 255)
        bdw[256] = part[255];
}

template <typename K, int BITS>
void radix_pass(const K *kin, const uint32_t *vin, K *kout, uint32_t *vout, const uint64_t *dcount, uint64_t hcount,
                uint64_t cap, uint32_t shift, uint32_t *scratch, hipStream_t s, Unpack un = Unpack{})
{
    hipLaunchKernelGGL((k_radix_hist<K, BITS>), dim3(kRadixBlocks), dim3(256), 0, s, kin, dcount, hcount, cap, shift,
                       scratch);
    hipLaunchKernelGGL(k_scan_rows, dim3((1 << BITS) / 16), dim3(1024), 0, s, scratch,
                       scratch + ((size_t)(1 << BITS) << kRadixShift));
    hipLaunchKernelGGL((k_radix_scatter<K, BITS>), dim3(kRadixBlocks), dim3(64 * kScatterWaves), 0, s, kin, vin, kout, vout,
                       dcount, hcount, cap, shift, scratch, un);
}

}  // namespace

void launch_length_sort(const uint32_t *len, uint32_t n, uint32_t *perm, uint32_t *off, uint32_t *bdw,
                        uint32_t *scratch, hipStream_t s)
{
    radix_pass<uint32_t, 8>(len, nullptr, nullptr, perm, nullptr, n, n, 0, scratch, s);
    hipLaunchKernelGGL(k_bucket_tables, dim3(1), dim3(256), 0, s, scratch, n, off, bdw);
}

void launch_sort_unpack(uint64_t *keys, uint64_t *tmp, const uint64_t *count, uint64_t cap, uint32_t lo_bit,
                        uint32_t hi_bit, uint32_t wbits, uint32_t *triples, int pairs_only, uint32_t *scratch,
                        hipStream_t s)
{
    uint64_t *a = keys, *b = tmp;
    for (uint32_t shift = lo_bit; shift < hi_bit; shift += kSortBits) {
        const bool last = shift + kSortBits >= hi_bit;
        radix_pass<uint64_t, kSortBits>(a, nullptr, b, nullptr, count, 0, cap, shift, scratch, s,
                                        last ? Unpack{triples, wbits, pairs_only} : Unpack{});
        uint64_t *t = a;
        a = b;
        b = t;
    }
}

}  // namespace fpm
