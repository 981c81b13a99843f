// fpm_build.hip -- preprocessing kernels: symbol statistics and selection
// (Section 3: common / rare / mixed symbol sets), length bucketing into
// padded blocks, and fingerprint construction (Section 3.2).
#include "fpm_internal.hpp"

namespace fpm {

namespace {

__global__ void k_zero(uint32_t *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_lengths(const uint64_t *offsets, uint32_t n, uint32_t *len_out, uint32_t *err)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t a = offsets[i], b = offsets[i + 1];
    uint32_t L;
    if (b < a) {
        atomicOr(err, 2u);
        L = 0;
    } else if (b - a > (uint64_t)kMaxLen) {
        atomicOr(err, 1u);
        L = kMaxLen;
    } else {
        L = (uint32_t)(b - a);
    }
    len_out[i] = L;
}

// Byte histogram of every string's bytes (the CSR range offsets[0] ..
// offsets[n]).  The aligned middle of the range is read 16 bytes per thread
// and load; each block counts into eight LDS copies of the histogram (copy =
// thread index mod 8), so lanes that meet the same frequent symbol mostly
// hit different copies instead of serialising on one address; the copies
// are summed into the 64-bit device histogram once per block.
constexpr uint32_t kHistCopies = 8;

__device__ __forceinline__ void hist_dword(uint32_t *h, uint32_t w)
{
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
        atomicAdd(&h[(w >> (8 * j)) & 0xFFu], 1u);
}

__global__ void __launch_bounds__(256) k_byte_hist(const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                                                   unsigned long long *hist)
{
    __shared__ uint32_t h[kHistCopies][257];  // padded: copies of one bin in different banks
    for (uint32_t i = threadIdx.x; i < kHistCopies * 257; i += blockDim.x)
        (&h[0][0])[i] = 0;
    __syncthreads();
    uint32_t *mine = h[threadIdx.x % kHistCopies];
    const uint64_t lo = offsets[0], hi = offsets[n];
    // [lo, a0): bytes before the first 16-byte aligned address; [a0, a1):
    // whole 16-byte groups; [a1, hi): the rest (each part of [lo, hi))
    const uint64_t skew = (16u - (((uintptr_t)bytes + lo) & 15u)) & 15u;
    const uint64_t a0 = lo + min(skew, hi - lo);
    const uint64_t a1 = a0 + ((hi - a0) & ~(uint64_t)15);
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    if (tid < a0 - lo)
        atomicAdd(&mine[bytes[lo + tid]], 1u);
    if (tid < hi - a1)
        atomicAdd(&mine[bytes[a1 + tid]], 1u);
    const uint4 *v = (const uint4 *)(bytes + a0);
    const uint64_t nv = (a1 - a0) >> 4;
    for (uint64_t g = tid; g < nv; g += nth) {
        const uint4 x = v[g];
        hist_dword(mine, x.x);
        hist_dword(mine, x.y);
        hist_dword(mine, x.z);
        hist_dword(mine, x.w);
    }
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (uint32_t c = 0; c < kHistCopies; ++c)
        t += h[c][threadIdx.x];
    if (t)
        atomicAdd(&hist[threadIdx.x], (unsigned long long)t);
}

// Symbol selection.  Thread c ranks byte c among the symbols that occur:
// descending rank orders by (count desc, byte asc), ascending rank by
// (count asc, byte asc).  common: field = descending rank < F; rare: field
// = ascending rank < F; mixed: the ceil(F/2) first in descending order, then
// the remaining symbols in ascending order until F fields are used.
__global__ void __launch_bounds__(256) k_select(const unsigned long long *hist, int nf, int symset, uint8_t *map)
{
    __shared__ unsigned long long h[256];
    __shared__ uint32_t rdesc[256];
    __shared__ uint32_t npresent;
    const uint32_t c = threadIdx.x;
    h[c] = hist[c];
    if (c == 0)
        npresent = 0;
    __syncthreads();
    const bool present = h[c] > 0;
    if (present)
        atomicAdd(&npresent, 1u);
    uint32_t rd = 0, ra = 0;
    for (uint32_t o = 0; o < 256; ++o) {
        if (h[o] == 0)
            continue;
        rd += (h[o] > h[c] || (h[o] == h[c] && o < c)) ? 1u : 0u;
        ra += (h[o] < h[c] || (h[o] == h[c] && o < c)) ? 1u : 0u;
    }
    rdesc[c] = present ? rd : 0xFFFFFFFFu;
    __syncthreads();
    uint32_t field = 0xFFu;
    if (present) {
        if (symset == 0) {
            if (rd < (uint32_t)nf)
                field = rd;
        } else if (symset == 1) {
            if (ra < (uint32_t)nf)
                field = ra;
        } else {
            const uint32_t hc = (uint32_t)(nf + 1) / 2;
            if (rd < hc) {
                field = rd;
            } else {
                const uint32_t ncommon = min(hc, npresent);
                uint32_t rr = 0;  // rank among the not-yet-chosen symbols, ascending order
                for (uint32_t o = 0; o < 256; ++o) {
                    if (h[o] == 0 || rdesc[o] < hc)
                        continue;
                    rr += (h[o] < h[c] || (h[o] == h[c] && o < c)) ? 1u : 0u;
                }
                if (ncommon + rr < (uint32_t)nf)
                    field = ncommon + rr;
            }
        }
    }
    map[c] = (uint8_t)field;
}

// A string whose slot would end beyond str_cap dwords (possible only when a
// caller's query bytes exceed the capacity it declared) becomes the empty
// string at offset 0 and err gets bit 4.
__global__ void k_layout(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit, const uint32_t *perm,
                         const uint32_t *len, const uint32_t *off, const uint32_t *bdw, uint32_t n, uint8_t *slen,
                         uint32_t *soff, uint32_t *str, uint64_t str_cap, uint32_t *err)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const uint32_t i = perm[p];
    uint32_t L = len[i];
    uint32_t sw = slot_dwords(L);
    uint32_t so = bdw[L] + (p - off[L]) * sw;
    if ((uint64_t)so + sw > str_cap) {
        atomicOr(err, 4u);
        slen[p] = 0;
        soff[p] = 0;
        return;
    }
    slen[p] = (uint8_t)L;
    soff[p] = so;
    const uint64_t start = offsets[i];
    const uint64_t end_all = offsets[n];
    const uint64_t limit = end_all < nbytes_limit ? end_all : nbytes_limit;
    for (uint32_t t = 0; t < sw; ++t) {
        uint32_t w = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t pos = 4 * t + j;
            const uint64_t a = start + pos;
            if (pos < L && a < limit)
                w |= (uint32_t)bytes[a] << (8 * j);
        }
        str[so + t] = w;
    }
}

// Fingerprint construction (Section 3.2), one dword (4 symbols) at a time.
// Field f of the map:
//   occ  -> bit f;
//   occh -> bit 2f for a symbol in the first floor(L/2) positions, 2f+1 after;
//   count-> 2-bit saturating counter at bits 2f, 2f+1;
//   pos  -> f < npos: first position (0-indexed) in 3 bits at 3f, all ones
//           when it is >= 7 or the symbol is absent; f >= npos: occurrence
//           bit 3*npos + (f - npos).
// Bigram fingerprints (VARIANT 4, the q-gram direction of Section 5) ignore
// the map: bigram (x, y) of the raw bytes sets bit
// ((x * 256 + y) * 2654435761 mod 2^32) >> (32 - log2(bits)) (Knuth's
// multiplicative hash).  Combined fingerprints (VARIANT 5, also Section 5):
// occurrence bit f in the low bits/2 bits and, for f < bits/4, a 2-bit
// saturating counter at bits/2 + 2f.  `aux` is log2(bits) for bigrams,
// bits/2 for combined and npos otherwise.
template <int VARIANT>
__device__ __forceinline__ uint32_t fp_init(uint32_t npos)
{
    if (VARIANT == 2)
        return (npos == 10) ? 0x3FFFFFFFu : 0x7FFFu;  // every position field starts at all ones
    return 0;
}

// Symbols 4t .. 4t+3 of a string of length L (held in w, first symbol in the
// low byte) into fp; prev carries the last symbol of the previous dword.
template <int VARIANT>
__device__ __forceinline__ void fp_dword(uint32_t &fp, uint32_t &prev, uint32_t w, uint32_t t, uint32_t L,
                                         const uint8_t *smap, uint32_t npos)
{
    const uint32_t half = L >> 1;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t pos = 4 * t + j;
        if (pos >= L)
            break;
        if (VARIANT == 4) {
            const uint32_t c = (w >> (8 * j)) & 0xFFu;
            if (pos > 0)
                fp |= 1u << (((prev * 256u + c) * 2654435761u) >> (32u - npos));
            prev = c;
            continue;
        }
        const uint32_t f = smap[(w >> (8 * j)) & 0xFFu];
        if (f == 0xFFu)
            continue;
        if (VARIANT == 5) {
            fp |= 1u << f;
            const uint32_t at = npos + 2 * f;
            if (f < npos / 2 && ((fp >> at) & 3u) != 3u)
                fp += 1u << at;
        } else if (VARIANT == 0) {
            fp |= 1u << f;
        } else if (VARIANT == 3) {
            fp |= 1u << (2 * f + (pos >= half ? 1u : 0u));
        } else if (VARIANT == 1) {
            if (((fp >> (2 * f)) & 3u) != 3u)
                fp += 1u << (2 * f);
        } else {
            if (f < npos) {
                if (pos < 7 && ((fp >> (3 * f)) & 7u) == 7u)
                    fp = (fp & ~(7u << (3 * f))) | (pos << (3 * f));
            } else {
                fp |= 1u << (3 * npos + (f - npos));
            }
        }
    }
}

template <int VARIANT>
__device__ __forceinline__ uint32_t fp_aux(int bits)
{
    return VARIANT == 4 ? (bits == 16 ? 4u : 5u) : VARIANT == 5 ? (uint32_t)bits / 2 : (uint32_t)bits / 3;
}

template <int VARIANT>
__device__ __forceinline__ uint32_t fingerprint(const uint32_t *s, uint32_t L, const uint8_t *smap, uint32_t npos)
{
    uint32_t fp = fp_init<VARIANT>(npos), prev = 0;
    const uint32_t nw = (L + 3) >> 2;
    for (uint32_t t = 0; t < nw; ++t)
        fp_dword<VARIANT>(fp, prev, s[t], t, L, smap, npos);
    return fp;
}

// Filter key of a fingerprint at sorted position p.
template <int VARIANT>
__device__ __forceinline__ void store_key(uint32_t fp, int key_kind, void *keys, uint32_t p, uint32_t aux)
{
    if (VARIANT == 1) {
        // thermometer expansion of each 2-bit count v: [v>=1, v>=2, v>=3];
        // the popcount of the XOR of two expansions is the L1 distance of
        // the counts.
        const uint32_t lo = fp & 0x55555555u, hi = (fp >> 1) & 0x55555555u;
        const uint32_t t0 = lo | hi, t1 = hi, t2 = lo & hi;
        if (key_is_64(key_kind)) {
            ((uint64_t *)keys)[p] = (uint64_t)(t0 | (t1 << 1)) | ((uint64_t)t2 << 32);
        } else {
            ((uint32_t *)keys)[p] = (t0 | (t1 << 1)) | (t2 << 16);  // 8 fields: bits 0..15 and 16..30
        }
    } else if (key_kind == kCombo64) {
        // occurrence half as it is (low word); the counters' thermometer
        // expansion (as for count keys) in the high word
        const uint32_t half = aux;  // bits / 2
        const uint32_t occ = fp & ((1u << half) - 1u), c = fp >> half;
        const uint32_t lo = c & 0x5555u, hi = (c >> 1) & 0x5555u;
        const uint32_t th = (lo | hi) | (hi << 1) | ((lo & hi) << 16);
        ((uint64_t *)keys)[p] = (uint64_t)occ | ((uint64_t)th << 32);
    } else if (key_kind == kTherm32) {
        // 16-bit fingerprint, thermometer code of its popcount above it
        ((uint32_t *)keys)[p] = fp | (((1u << __builtin_popcount(fp)) - 1u) << 16);
    } else {
        ((uint32_t *)keys)[p] = fp;
    }
}

template <int VARIANT>
__global__ void __launch_bounds__(256) k_fingerprints(const uint32_t *str, const uint32_t *soff, const uint8_t *slen,
                                                      const uint32_t *perm, uint32_t n, const uint8_t *map, int bits,
                                                      uint32_t *fp_sorted, uint32_t *fp_orig, void *keys,
                                                      int key_kind)
{
    __shared__ uint8_t smap[256];
    smap[threadIdx.x] = map[threadIdx.x];
    __syncthreads();
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const uint32_t aux = fp_aux<VARIANT>(bits);
    const uint32_t fp = fingerprint<VARIANT>(str + soff[p], slen[p], smap, aux);
    if (fp_sorted)
        fp_sorted[p] = fp;
    if (fp_orig)
        fp_orig[perm[p]] = fp;
    if (keys)
        store_key<VARIANT>(fp, key_kind, keys, p, aux);
}

// k_layout followed by the fingerprint of each string, built from the
// dwords as they are written (one pass over the bytes).  The string is read
// as the aligned source dwords that hold its bytes -- four loads in flight
// per step -- and each slot dword is funnel-shifted out of two neighbours
// (v_alignbyte); every dword read holds at least one byte of the string
// below the read limit, so no read leaves the pages of the input.
template <int VARIANT>
__global__ void __launch_bounds__(256) k_layout_fp(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit,
                                                   const uint32_t *perm, const uint32_t *len, const uint32_t *off,
                                                   const uint32_t *bdw, uint32_t n, uint8_t *slen, uint32_t *soff,
                                                   uint32_t *str, uint64_t str_cap, uint32_t *err, const uint8_t *map,
                                                   int bits, uint32_t *fp_orig, void *keys, int key_kind)
{
    __shared__ uint8_t smap[256];
    smap[threadIdx.x] = map[threadIdx.x];
    __syncthreads();
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const uint32_t npos = fp_aux<VARIANT>(bits);
    uint32_t fp = fp_init<VARIANT>(npos), prev = 0;
    const uint32_t i = perm[p];
    const uint32_t L = len[i];
    const uint32_t sw = slot_dwords(L);
    const uint32_t so = bdw[L] + (p - off[L]) * sw;
    if ((uint64_t)so + sw > str_cap) {
        atomicOr(err, 4u);
        slen[p] = 0;
        soff[p] = 0;
    } else {
        slen[p] = (uint8_t)L;
        soff[p] = so;
        const uint64_t start = offsets[i];
        const uint64_t end_all = offsets[n];
        const uint64_t limit = end_all < nbytes_limit ? end_all : nbytes_limit;
        // bytes of the string below the read limit; the rest of the slot is zero
        const uint32_t le = start >= limit ? 0u : (uint32_t)min((uint64_t)L, limit - start);
        const uintptr_t a0 = (uintptr_t)(bytes + start);
        const uint32_t *src = (const uint32_t *)(a0 & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a0 & 3u);
        const uint32_t nsrc = (sh + le + 3u) >> 2;  // source dwords holding bytes of the string
        uint32_t cur = nsrc ? src[0] : 0u;
        for (uint32_t t = 0; t < sw; t += 4) {
            uint32_t nx[4], w[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u)
                nx[u] = (t + u + 1 < nsrc) ? src[t + u + 1] : 0u;
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t lo = u ? nx[u - 1] : cur;
                const int rem = (int)le - 4 * (int)(t + u);
                const uint32_t m = rem >= 4 ? ~0u : (rem <= 0 ? 0u : (1u << (8u * (uint32_t)rem)) - 1u);
                w[u] = __builtin_amdgcn_alignbyte(nx[u], lo, sh) & m;
            }
            cur = nx[3];
            if (sw >= 4) {  // whole 16-byte groups (slots of 4 ceil(L / 16) dwords, 16-byte aligned)
                *(uint4 *)(str + so + t) = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u)
                    fp_dword<VARIANT>(fp, prev, w[u], t + u, L, smap, npos);
            } else {  // L <= 8: one or two dwords
                str[so] = w[0];
                fp_dword<VARIANT>(fp, prev, w[0], 0, L, smap, npos);
                if (sw > 1) {
                    str[so + 1] = w[1];
                    fp_dword<VARIANT>(fp, prev, w[1], 1, L, smap, npos);
                }
            }
        }
    }
    if (fp_orig)
        fp_orig[i] = fp;
    store_key<VARIANT>(fp, key_kind, keys, p, npos);
}

// Reorder a laid-out set inside its length blocks by key popcount (stable):
// one block of kOrderWaves waves per length L, each wave owning a contiguous
// part of the length block.  Pass 1 counts each part's popcounts in LDS; the
// counts are turned into each wave's first destination per popcount; pass 2
// walks each part 64 positions at a time, ranks a lane among the lanes of
// equal popcount with 7 ballots, and moves the padded string (the slot size
// is uniform in a block), the caller index and the key to the new position.
// Popcounts are at most 64.
constexpr int kOrderWaves = 16;

__global__ void __launch_bounds__(64 * kOrderWaves) k_pop_order(const uint32_t *off, const uint32_t *bdw,
                                                                const uint32_t *str, const uint32_t *perm,
                                                                const void *keys, int key_kind, uint32_t *str_out,
                                                                uint32_t *perm_out, void *keys_out)
{
    __shared__ uint32_t run[kOrderWaves][65];
    __shared__ uint32_t base[65];
    const uint32_t L = blockIdx.x, lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t s = off[L], e = off[L + 1];
    if (s == e)
        return;
    const bool wide = key_is_64(key_kind);
    const uint64_t *k64 = (const uint64_t *)keys;
    const uint32_t *k32 = (const uint32_t *)keys;
    for (uint32_t i = threadIdx.x; i < kOrderWaves * 65; i += blockDim.x)
        (&run[0][0])[i] = 0;
    __syncthreads();
    const uint32_t lo = s + (uint32_t)((uint64_t)(e - s) * w / kOrderWaves);
    const uint32_t hi = s + (uint32_t)((uint64_t)(e - s) * (w + 1) / kOrderWaves);
    for (uint32_t i = lo + lane; i < hi; i += 64)
        atomicAdd(&run[w][wide ? __popcll(k64[i]) : __builtin_popcount(k32[i])], 1u);
    __syncthreads();
    if (threadIdx.x < 65) {
        uint32_t t = 0;
        for (int ww = 0; ww < kOrderWaves; ++ww)
            t += run[ww][threadIdx.x];
        base[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = s;
        for (int b = 0; b < 65; ++b) {
            const uint32_t c = base[b];
            base[b] = acc;
            acc += c;
        }
    }
    __syncthreads();
    if (threadIdx.x < 65) {
        uint32_t acc = base[threadIdx.x];
        for (int ww = 0; ww < kOrderWaves; ++ww) {
            const uint32_t c = run[ww][threadIdx.x];
            run[ww][threadIdx.x] = acc;
            acc += c;
        }
    }
    __syncthreads();
    const uint32_t sw = slot_dwords(L);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t *running = run[w];
    for (uint32_t c0 = lo; c0 < hi; c0 += 64) {
        const uint32_t i = c0 + lane;
        const bool active = i < hi;
        uint64_t kv = 0;
        if (active)
            kv = wide ? k64[i] : k32[i];
        const uint32_t pop = (uint32_t)__popcll(kv);
        uint64_t peers = __ballot(active);
#pragma unroll
        for (int bit = 0; bit < 7; ++bit) {
            const bool set = (pop >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t start = running[pop];
        __builtin_amdgcn_wave_barrier();
        if (active) {
            const uint32_t rank = (uint32_t)__popcll(peers & below);
            const uint32_t np = start + rank;
            const uint32_t *in = str + bdw[L] + (i - s) * sw;
            uint32_t *out = str_out + bdw[L] + (np - s) * sw;
            for (uint32_t t = 0; t < sw; ++t)
                out[t] = in[t];
            perm_out[np] = perm[i];
            if (wide)
                ((uint64_t *)keys_out)[np] = kv;
            else
                ((uint32_t *)keys_out)[np] = (uint32_t)kv;
            if (rank == 0)
                running[pop] = start + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void k_invert(const uint32_t *perm, uint32_t n, uint32_t *inv)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n)
        inv[perm[p]] = p;
}

inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

}  // namespace

void launch_zero(void *p, size_t n_u32, hipStream_t s)
{
    if (n_u32 == 0)
        return;
    uint32_t blocks = (uint32_t)std::min<size_t>(1024, (n_u32 + 255) / 256);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, n_u32);
}

void launch_lengths(const uint64_t *offsets, uint32_t n, uint32_t *len_out, uint32_t *err, hipStream_t s)
{
    if (n == 0)
        return;
    hipLaunchKernelGGL(k_lengths, dim3(blocks_for(n, 256)), dim3(256), 0, s, offsets, n, len_out, err);
}

void launch_byte_histogram(const uint8_t *bytes, const uint64_t *offsets, uint32_t n, unsigned long long *hist,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_byte_hist, dim3(1024), dim3(256), 0, s, bytes, offsets, n, hist);
}

void launch_select_symbols(const unsigned long long *hist, int nfields, int symset, uint8_t *map_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_select, dim3(1), dim3(256), 0, s, hist, nfields, symset, map_out);
}

void launch_layout(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit, const uint32_t *perm,
                   const uint32_t *len, const uint32_t *off, const uint32_t *bdw, uint32_t n, uint8_t *slen,
                   uint32_t *soff, uint32_t *str, uint64_t str_cap, uint32_t *err, hipStream_t s)
{
    if (n == 0)
        return;
    hipLaunchKernelGGL(k_layout, dim3(blocks_for(n, 256)), dim3(256), 0, s, bytes, offsets, nbytes_limit, perm, len,
                       off, bdw, n, slen, soff, str, str_cap, err);
}

void launch_layout_fp(const uint8_t *bytes, const uint64_t *offsets, uint64_t nbytes_limit, const uint32_t *perm,
                      const uint32_t *len, const uint32_t *off, const uint32_t *bdw, uint32_t n, uint8_t *slen,
                      uint32_t *soff, uint32_t *str, uint64_t str_cap, uint32_t *err, const uint8_t *map, int variant,
                      int bits, uint32_t *fp_orig, void *keys, int key_kind, hipStream_t s)
{
    if (n == 0)
        return;
    dim3 g(blocks_for(n, 256)), b(256);
#define FPM_LAYOUT_FP(V)                                                                                              \
    hipLaunchKernelGGL(k_layout_fp<V>, g, b, 0, s, bytes, offsets, nbytes_limit, perm, len, off, bdw, n, slen, soff,  \
                       str, str_cap, err, map, bits, fp_orig, keys, key_kind)
    switch (variant) {
    case 0:
        FPM_LAYOUT_FP(0);
        break;
    case 1:
        FPM_LAYOUT_FP(1);
        break;
    case 2:
        FPM_LAYOUT_FP(2);
        break;
    case 3:
        FPM_LAYOUT_FP(3);
        break;
    case 4:
        FPM_LAYOUT_FP(4);
        break;
    default:
        FPM_LAYOUT_FP(5);
        break;
    }
#undef FPM_LAYOUT_FP
}

void launch_fingerprints(const uint32_t *str, const uint32_t *soff, const uint8_t *slen, const uint32_t *perm,
                         uint32_t n, const uint8_t *map, int variant, int bits, uint32_t *fp_sorted,
                         uint32_t *fp_orig, void *keys, int key_kind, hipStream_t s)
{
    if (n == 0)
        return;
    dim3 g(blocks_for(n, 256)), b(256);
#define FPM_FINGERPRINTS(V)                                                                                           \
    hipLaunchKernelGGL(k_fingerprints<V>, g, b, 0, s, str, soff, slen, perm, n, map, bits, fp_sorted, fp_orig, keys,  \
                       key_kind)
    switch (variant) {
    case 0:
        FPM_FINGERPRINTS(0);
        break;
    case 1:
        FPM_FINGERPRINTS(1);
        break;
    case 2:
        FPM_FINGERPRINTS(2);
        break;
    case 3:
        FPM_FINGERPRINTS(3);
        break;
    case 4:
        FPM_FINGERPRINTS(4);
        break;
    default:
        FPM_FINGERPRINTS(5);
        break;
    }
#undef FPM_FINGERPRINTS
}

void launch_pop_order(const uint32_t *off, const uint32_t *bdw, const uint32_t *str, const uint32_t *perm,
                      const void *keys, int key_kind, uint32_t *str_out, uint32_t *perm_out, void *keys_out,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_pop_order, dim3(256), dim3(64 * kOrderWaves), 0, s, off, bdw, str, perm, keys, key_kind,
                       str_out, perm_out, keys_out);
}

void launch_invert(const uint32_t *perm, uint32_t n, uint32_t *inv, hipStream_t s)
{
    if (n == 0)
        return;
    hipLaunchKernelGGL(k_invert, dim3(blocks_for(n, 256)), dim3(256), 0, s, perm, n, inv);
}

}  // namespace fpm
