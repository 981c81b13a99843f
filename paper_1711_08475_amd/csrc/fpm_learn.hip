// fpm_learn.hip -- learned symbol-to-field grouping for occurrence
// fingerprints: FP32 training kernels (MLP forward, expected-F_D pair loss
// and its gradient, MLP backward, Adam) and the native training loop behind
// fpm_learn_grouping / fpm_learn_step (declared in fpm_learn.h).
//
// Model, per symbol c (one row of X):
//   pre = x_c W1 + b1, h = relu(pre), z = h W2 + b2, P_c = softmax(z)
// over B fields and a final "no field" column.  With L_cj = log(1 - P_cj),
// a string with symbol set S leaves bit j clear with probability
// Z_S,j = exp(sum_{c in S} L_cj) when every symbol independently picks its
// field from P_c; a pair (A, B) then has expected F_D
//   E = sum_j Z_A,j + Z_B,j - 2 Z_{A u B},j
// (bit j differs iff exactly one side has it).  Loss per non-matching pair:
// softplus(beta (t - E)) / beta with t = 2k + 1 + margin.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/fpm_learn.h"
#include "fpm_host.hpp"
#include "fpm_internal.hpp"

using namespace fpm;

namespace {

constexpr int kMaxSym = 128;
constexpr int kMaxHidden = 128;
constexpr float kPClamp = 1e-7f;  // 1 - P is clamped below at this value

struct Shapes {
    uint32_t sigma, d_in, hidden, bits;
    __host__ __device__ uint32_t n_w1() const { return d_in * hidden; }
    __host__ __device__ uint32_t n_w2() const { return hidden * (bits + 1); }
    __host__ __device__ uint32_t n_params() const { return n_w1() + hidden + n_w2() + bits + 1; }
};

// ------------------------------------------------------------------ kernels

// Symbol set of each string as a 128-bit mask over model symbols.
__global__ void k_symbol_masks(const uint8_t *bytes, const uint64_t *offsets, uint32_t n, const uint8_t *sym_index,
                               uint64_t *masks)
{
    __shared__ uint8_t sidx[256];
    sidx[threadIdx.x] = sym_index[threadIdx.x];
    __syncthreads();
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t lo = 0, hi = 0;
    for (uint64_t t = offsets[i]; t < offsets[i + 1]; ++t) {
        const uint32_t s = sidx[bytes[t]];
        if (s < 64)
            lo |= 1ull << s;
        else if (s < 128)
            hi |= 1ull << (s - 64);
    }
    masks[2 * i] = lo;
    masks[2 * i + 1] = hi;
}

// Pair masks for a batch: ma / mb get the query / word masks of each
// non-matching pair.
__global__ void k_gather_pair_masks(const uint32_t *pairs, uint64_t n, const uint64_t *qmask, const uint64_t *dmask,
                                    uint64_t *ma, uint64_t *mb)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t q = pairs[2 * i], w = pairs[2 * i + 1];
    ma[2 * i] = qmask[2 * q];
    ma[2 * i + 1] = qmask[2 * q + 1];
    mb[2 * i] = dmask[2 * w];
    mb[2 * i + 1] = dmask[2 * w + 1];
}

// MLP forward: one block per symbol row.
__global__ void __launch_bounds__(128) k_mlp_forward(const float *X, const float *params, Shapes sh, float *pre,
                                                     float *hid, float *P, float *L)
{
    __shared__ float sh_h[kMaxHidden];
    __shared__ float sh_z[kMaxHidden];
    const uint32_t c = blockIdx.x, t = threadIdx.x;
    const float *W1 = params, *b1 = W1 + sh.n_w1(), *W2 = b1 + sh.hidden, *b2 = W2 + sh.n_w2();
    const uint32_t nb = sh.bits + 1;
    if (t < sh.hidden) {
        float a = b1[t];
        for (uint32_t i = 0; i < sh.d_in; ++i)
            a += X[c * sh.d_in + i] * W1[i * sh.hidden + t];
        pre[c * sh.hidden + t] = a;
        const float h = a > 0.f ? a : 0.f;
        hid[c * sh.hidden + t] = h;
        sh_h[t] = h;
    }
    __syncthreads();
    if (t < nb) {
        float z = b2[t];
        for (uint32_t h = 0; h < sh.hidden; ++h)
            z += sh_h[h] * W2[h * nb + t];
        sh_z[t] = z;
    }
    __syncthreads();
    if (t < nb) {
        float mx = sh_z[0];
        for (uint32_t j = 1; j < nb; ++j)
            mx = fmaxf(mx, sh_z[j]);
        float den = 0.f;
        for (uint32_t j = 0; j < nb; ++j)
            den += expf(sh_z[j] - mx);
        const float p = expf(sh_z[t] - mx) / den;
        P[c * nb + t] = p;
        if (t < sh.bits)
            L[c * sh.bits + t] = logf(fmaxf(1.f - p, kPClamp));
    }
}

// Pair loss and dLoss/dL.  B lanes per pair, lane j owns field j; G gets the
// sum over pairs of dloss/dL_cj (unnormalised), sums[0] the summed pair
// loss, sums[1] the summed expected F_D.
template <int B>
__global__ void __launch_bounds__(256) k_pair_loss(const float *L, const uint64_t *ma, const uint64_t *mb, uint64_t n,
                                                   uint32_t sigma, float target, float beta, float *G, float *sums)
{
    __shared__ float sL[kMaxSym * B];
    __shared__ float sG[kMaxSym * B];
    __shared__ float sred[2];
    for (uint32_t i = threadIdx.x; i < sigma * B; i += blockDim.x) {
        sL[i] = L[i];
        sG[i] = 0.f;
    }
    if (threadIdx.x < 2)
        sred[threadIdx.x] = 0.f;
    __syncthreads();
    const uint32_t j = threadIdx.x % B;
    const uint32_t groups = blockDim.x / B;
    float loss_acc = 0.f, e_acc = 0.f;
    for (uint64_t p = blockIdx.x * (uint64_t)groups + threadIdx.x / B; p < n; p += (uint64_t)gridDim.x * groups) {
        const uint64_t a0 = ma[2 * p], a1 = ma[2 * p + 1], b0 = mb[2 * p], b1 = mb[2 * p + 1];
        float ua = 0.f, ub = 0.f, uab = 0.f;
        for (int half = 0; half < 2; ++half) {
            uint64_t u = half ? (a1 | b1) : (a0 | b0);
            const uint64_t am = half ? a1 : a0, bm = half ? b1 : b0;
            while (u) {
                const uint32_t bit = (uint32_t)__builtin_ctzll(u);
                u &= u - 1;
                const float l = sL[(bit + 64 * half) * B + j];
                uab += l;
                if ((am >> bit) & 1ull)
                    ua += l;
                if ((bm >> bit) & 1ull)
                    ub += l;
            }
        }
        const float za = expf(ua), zb = expf(ub), zab = expf(uab);
        float e = za + zb - 2.f * zab;
#pragma unroll
        for (int o = B / 2; o >= 1; o >>= 1)
            e += __shfl_xor(e, o, B);
        const float x = beta * (target - e);
        const float sp = x > 20.f ? x : log1pf(expf(x));  // softplus
        const float s = -1.f / (1.f + expf(-x));           // d loss / d E
        if (j == 0) {
            loss_acc += sp / beta;
            e_acc += e;
        }
        for (int half = 0; half < 2; ++half) {
            uint64_t u = half ? (a1 | b1) : (a0 | b0);
            const uint64_t am = half ? a1 : a0, bm = half ? b1 : b0;
            while (u) {
                const uint32_t bit = (uint32_t)__builtin_ctzll(u);
                u &= u - 1;
                float g = -2.f * zab;
                if ((am >> bit) & 1ull)
                    g += za;
                if ((bm >> bit) & 1ull)
                    g += zb;
                atomicAdd(&sG[(bit + 64 * half) * B + j], s * g);
            }
        }
    }
    atomicAdd(&sred[0], loss_acc);
    atomicAdd(&sred[1], e_acc);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < sigma * B; i += blockDim.x)
        if (sG[i] != 0.f)
            atomicAdd(&G[i], sG[i]);
    if (threadIdx.x == 0) {
        atomicAdd(&sums[0], sred[0]);
        atomicAdd(&sums[1], sred[1]);
    }
}

// MLP backward, one block.  G holds the summed pair gradient dloss/dL; it is
// divided by npairs; the entropy term adds ew * mean_c H(P_c).  sums[2]
// receives the mean entropy.
__global__ void __launch_bounds__(256) k_mlp_backward(const float *X, const float *params, Shapes sh,
                                                      const float *pre, const float *hid, const float *P,
                                                      const float *G, float npairs, float ew, float *grads,
                                                      float *sums, float *dh)
{
    __shared__ float dz[kMaxSym * 33];  // sigma x (bits + 1); dh (sigma x hidden) is global scratch
    const uint32_t nb = sh.bits + 1;
    __shared__ float ent_acc;
    const float *W1 = params, *b1 = W1 + sh.n_w1(), *W2 = b1 + sh.hidden;
    (void)b1;
    float *gW1 = grads, *gb1 = gW1 + sh.n_w1(), *gW2 = gb1 + sh.hidden, *gb2 = gW2 + sh.n_w2();
    const float inv = npairs > 0.f ? 1.f / npairs : 0.f;
    const float went = ew / (float)sh.sigma;
    if (threadIdx.x == 0)
        ent_acc = 0.f;
    __syncthreads();
    // dloss/dz for every symbol row (softmax backward)
    for (uint32_t c = threadIdx.x; c < sh.sigma; c += blockDim.x) {
        float dot = 0.f, ent = 0.f;
        for (uint32_t j = 0; j < nb; ++j) {
            const float p = P[c * nb + j];
            float g = 0.f;
            if (j < sh.bits)
                g = G[c * sh.bits + j] * inv * (-1.f / fmaxf(1.f - p, kPClamp));
            const float lp = logf(fmaxf(p, 1e-30f));
            g += went * (-(lp + 1.f));
            ent -= p * lp;
            dz[c * nb + j] = g;
            dot += p * g;
        }
        for (uint32_t j = 0; j < nb; ++j)
            dz[c * nb + j] = P[c * nb + j] * (dz[c * nb + j] - dot);
        atomicAdd(&ent_acc, ent);
    }
    __syncthreads();
    // W2, b2
    for (uint32_t e = threadIdx.x; e < sh.hidden * nb; e += blockDim.x) {
        const uint32_t h = e / nb, j = e % nb;
        float a = 0.f;
        for (uint32_t c = 0; c < sh.sigma; ++c)
            a += hid[c * sh.hidden + h] * dz[c * nb + j];
        gW2[e] = a;
    }
    for (uint32_t j = threadIdx.x; j < nb; j += blockDim.x) {
        float a = 0.f;
        for (uint32_t c = 0; c < sh.sigma; ++c)
            a += dz[c * nb + j];
        gb2[j] = a;
    }
    // hidden layer
    for (uint32_t e = threadIdx.x; e < sh.sigma * sh.hidden; e += blockDim.x) {
        const uint32_t c = e / sh.hidden, h = e % sh.hidden;
        float a = 0.f;
        if (pre[e] > 0.f)
            for (uint32_t j = 0; j < nb; ++j)
                a += dz[c * nb + j] * W2[h * nb + j];
        dh[e] = a;
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < sh.d_in * sh.hidden; e += blockDim.x) {
        const uint32_t i = e / sh.hidden, h = e % sh.hidden;
        float a = 0.f;
        for (uint32_t c = 0; c < sh.sigma; ++c)
            a += X[c * sh.d_in + i] * dh[c * sh.hidden + h];
        gW1[e] = a;
    }
    for (uint32_t h = threadIdx.x; h < sh.hidden; h += blockDim.x) {
        float a = 0.f;
        for (uint32_t c = 0; c < sh.sigma; ++c)
            a += dh[c * sh.hidden + h];
        gb1[h] = a;
    }
    if (threadIdx.x == 0)
        sums[2] = ent_acc / (float)sh.sigma;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fill(float *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.f;
}

// ---------------------------------------------------------------- host side

struct Model {
    Shapes sh{};
    float *X = nullptr, *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    float *pre = nullptr, *hid = nullptr, *P = nullptr, *L = nullptr, *G = nullptr, *sums = nullptr;
    float *dh = nullptr;
    ~Model()
    {
        dfree(X);
        dfree(params);
        dfree(grads);
        dfree(m);
        dfree(v);
        dfree(pre);
        dfree(hid);
        dfree(P);
        dfree(L);
        dfree(G);
        dfree(sums);
        dfree(dh);
    }
    hipError_t alloc(const Shapes &s)
    {
        sh = s;
        hipError_t e;
        const uint32_t np = s.n_params();
        if ((e = dalloc(&X, (size_t)s.sigma * s.d_in)) || (e = dalloc(&params, np)) || (e = dalloc(&grads, np)) ||
            (e = dalloc(&m, np)) || (e = dalloc(&v, np)) || (e = dalloc(&pre, (size_t)s.sigma * s.hidden)) ||
            (e = dalloc(&hid, (size_t)s.sigma * s.hidden)) || (e = dalloc(&P, (size_t)s.sigma * (s.bits + 1))) ||
            (e = dalloc(&L, (size_t)s.sigma * s.bits)) || (e = dalloc(&G, (size_t)s.sigma * s.bits)) ||
            (e = dalloc(&sums, 4)) || (e = dalloc(&dh, (size_t)s.sigma * s.hidden)))
            return e;
        return hipSuccess;
    }
};

void launch_fill(float *p, uint32_t n, hipStream_t s)
{
    if (n)
        hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

// forward + pair loss + backward on a batch of pair masks
hipError_t forward_backward(Model &M, const uint64_t *ma, const uint64_t *mb, uint64_t n, float target, float beta,
                            float ew, hipStream_t s)
{
    const Shapes &sh = M.sh;
    launch_fill(M.G, sh.sigma * sh.bits, s);
    launch_fill(M.sums, 4, s);
    hipLaunchKernelGGL(k_mlp_forward, dim3(sh.sigma), dim3(128), 0, s, M.X, M.params, sh, M.pre, M.hid, M.P, M.L);
    if (n) {
        const uint32_t groups = 256 / sh.bits;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(2048, (n + groups - 1) / groups);
        if (sh.bits == 16)
            hipLaunchKernelGGL(k_pair_loss<16>, dim3(blocks), dim3(256), 0, s, M.L, ma, mb, n, sh.sigma, target, beta,
                               M.G, M.sums);
        else
            hipLaunchKernelGGL(k_pair_loss<32>, dim3(blocks), dim3(256), 0, s, M.L, ma, mb, n, sh.sigma, target, beta,
                               M.G, M.sums);
    }
    hipLaunchKernelGGL(k_mlp_backward, dim3(1), dim3(256), 0, s, M.X, M.params, sh, M.pre, M.hid, M.P, M.G,
                       (float)n, ew, M.grads, M.sums, M.dh);
    return hipGetLastError();
}

fpm_status check_shapes(const Shapes &sh)
{
    if (sh.bits != 16 && sh.bits != 32)
        return fail(FPM_EINVAL, "learned grouping: bits must be 16 or 32");
    if (sh.sigma == 0 || sh.sigma > (uint32_t)kMaxSym)
        return fail(FPM_EINVAL, "learned grouping: 1..%d symbols", kMaxSym);
    if (sh.hidden == 0 || sh.hidden > (uint32_t)kMaxHidden)
        return fail(FPM_EINVAL, "learned grouping: hidden width 1..%d", kMaxHidden);
    if (sh.d_in == 0 || sh.d_in > 1024)
        return fail(FPM_EINVAL, "learned grouping: 1..1024 features");
    return FPM_OK;
}

}  // namespace

extern "C" {

fpm_status fpm_learn_step(uint32_t sigma, uint32_t d_in, uint32_t hidden, uint32_t bits, uint32_t k, const float *X,
                          const float *params, const uint64_t *masks_a, const uint64_t *masks_b, uint64_t n_pairs,
                          float margin, float beta, float entropy_weight, float *P_out, float *loss_out,
                          float *grads_out)
{
    g_last_error.clear();
    Shapes sh{sigma, d_in, hidden, bits};
    fpm_status st = check_shapes(sh);
    if (st)
        return st;
    if (!X || !params || !P_out || !loss_out || !grads_out || (n_pairs && (!masks_a || !masks_b)))
        return fail(FPM_EINVAL, "null pointer");
    if (k < 1 || k > 2)
        return fail(FPM_EUNSUPPORTED, "k must be 1 or 2");
    Model M;
    uint64_t *ma = nullptr, *mb = nullptr;
    hipError_t e;
    if ((e = M.alloc(sh)) || (e = dalloc(&ma, 2 * n_pairs)) || (e = dalloc(&mb, 2 * n_pairs))) {
        dfree(ma);
        dfree(mb);
        return hip_fail(e, "fpm_learn_step alloc");
    }
    hipStream_t s = nullptr;
    (void)hipMemcpy(M.X, X, sizeof(float) * sigma * d_in, hipMemcpyHostToDevice);
    (void)hipMemcpy(M.params, params, sizeof(float) * sh.n_params(), hipMemcpyHostToDevice);
    if (n_pairs) {
        (void)hipMemcpy(ma, masks_a, sizeof(uint64_t) * 2 * n_pairs, hipMemcpyHostToDevice);
        (void)hipMemcpy(mb, masks_b, sizeof(uint64_t) * 2 * n_pairs, hipMemcpyHostToDevice);
    }
    e = forward_backward(M, ma, mb, n_pairs, (float)(2 * k + 1) + margin, beta, entropy_weight, s);
    float sums[4] = {0, 0, 0, 0};
    if (!e)
        e = hipMemcpy(P_out, M.P, sizeof(float) * sigma * (bits + 1), hipMemcpyDeviceToHost);
    if (!e)
        e = hipMemcpy(grads_out, M.grads, sizeof(float) * sh.n_params(), hipMemcpyDeviceToHost);
    if (!e)
        e = hipMemcpy(sums, M.sums, sizeof(sums), hipMemcpyDeviceToHost);
    dfree(ma);
    dfree(mb);
    if (e)
        return hip_fail(e, "fpm_learn_step");
    const float inv = n_pairs ? 1.f / (float)n_pairs : 0.f;
    loss_out[0] = sums[0] * inv;
    loss_out[1] = sums[2];
    loss_out[2] = sums[1] * inv;
    return FPM_OK;
}

fpm_status fpm_learn_grouping(const uint8_t *dbytes, const uint64_t *doffsets, uint32_t n_words,
                              const uint8_t *qbytes, const uint64_t *qoffsets, uint32_t n_queries,
                              const uint32_t *pairs, const uint8_t *is_match, uint64_t n_pairs,
                              const fpm_learn_config *cfg_in, uint8_t map_out[256], fpm_learn_report *report)
{
    g_last_error.clear();
    if (!dbytes || !doffsets || !qbytes || !qoffsets || !map_out || (n_pairs && (!pairs || !is_match)))
        return fail(FPM_EINVAL, "null pointer");
    fpm_learn_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    if (cfg_in)
        cfg = *cfg_in;
    if (!cfg.bits)
        cfg.bits = 16;
    if (!cfg.k)
        cfg.k = 1;
    if (!cfg.hidden)
        cfg.hidden = 64;
    if (!cfg.epochs)
        cfg.epochs = 40;
    if (!cfg.batch)
        cfg.batch = 65536;
    if (cfg.lr <= 0.f)
        cfg.lr = 0.01f;
    if (cfg.beta <= 0.f)
        cfg.beta = 2.f;
    if (cfg.margin < 0.f)
        cfg.margin = 0.f;
    if (cfg.k > 2)
        return fail(FPM_EUNSUPPORTED, "k must be 1 or 2");
    for (uint64_t i = 0; i < n_pairs; ++i)
        if (pairs[2 * i] >= n_queries || pairs[2 * i + 1] >= n_words)
            return fail(FPM_EINVAL, "pair %llu out of range", (unsigned long long)i);
    for (uint32_t i = 0; i < n_words; ++i)
        if (doffsets[i + 1] < doffsets[i])
            return fail(FPM_EINVAL, "dictionary offsets decrease");
    for (uint32_t i = 0; i < n_queries; ++i)
        if (qoffsets[i + 1] < qoffsets[i])
            return fail(FPM_EINVAL, "query offsets decrease");

    // symbol statistics on the host (features only; the fingerprint
    // alphabet itself comes from the GPU byte histogram below)
    const uint64_t dn = doffsets[n_words], qn = qoffsets[n_queries];
    std::vector<double> cnt(256, 0.0), words_with(256, 0.0), relpos(256, 0.0);
    {
        std::vector<uint32_t> last_seen(256, 0xFFFFFFFFu);
        for (uint32_t w = 0; w < n_words; ++w) {
            const uint64_t a = doffsets[w], b = doffsets[w + 1];
            const double len = (double)(b - a);
            for (uint64_t t = a; t < b; ++t) {
                const uint8_t c = dbytes[t];
                cnt[c] += 1.0;
                relpos[c] += len > 1 ? (double)(t - a) / (len - 1) : 0.5;
                if (last_seen[c] != w) {
                    last_seen[c] = w;
                    words_with[c] += 1.0;
                }
            }
        }
    }
    std::vector<int> syms;
    for (int c = 0; c < 256; ++c)
        if (cnt[c] > 0)
            syms.push_back(c);
    std::stable_sort(syms.begin(), syms.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
    if (syms.size() > (size_t)kMaxSym)
        syms.resize(kMaxSym);
    Shapes sh{(uint32_t)syms.size(), (uint32_t)syms.size() + 4, cfg.hidden, cfg.bits};
    if (sh.sigma == 0) {
        memset(map_out, 0xFF, 256);
        return FPM_OK;
    }
    fpm_status st = check_shapes(sh);
    if (st)
        return st;
    uint8_t sym_index[256];
    memset(sym_index, 0xFF, sizeof(sym_index));
    std::vector<float> X((size_t)sh.sigma * sh.d_in, 0.f);
    const double maxlog = std::log(cnt[syms[0]] + 1.0);
    for (uint32_t s = 0; s < sh.sigma; ++s) {
        const int c = syms[s];
        sym_index[c] = (uint8_t)s;
        float *x = &X[(size_t)s * sh.d_in];
        x[s] = 1.f;
        x[sh.sigma + 0] = (float)(std::log(cnt[c] + 1.0) / maxlog);
        x[sh.sigma + 1] = (float)s / (float)sh.sigma;
        x[sh.sigma + 2] = n_words ? (float)(words_with[c] / n_words) : 0.f;
        x[sh.sigma + 3] = (float)(relpos[c] / cnt[c]);
    }
    // seeded initialisation
    std::vector<float> params(sh.n_params(), 0.f);
    {
        std::mt19937_64 rng(cfg.seed ? cfg.seed : 0x5eed);
        std::normal_distribution<float> nd(0.f, 1.f);
        const float s1 = 1.f / std::sqrt((float)sh.d_in), s2 = 1.f / std::sqrt((float)sh.hidden);
        for (uint32_t i = 0; i < sh.n_w1(); ++i)
            params[i] = nd(rng) * s1;
        float *w2 = &params[sh.n_w1() + sh.hidden];
        for (uint32_t i = 0; i < sh.n_w2(); ++i)
            w2[i] = nd(rng) * s2;
    }
    // training pairs: the non-matching ones
    std::vector<uint32_t> tp;
    tp.reserve(2 * n_pairs);
    for (uint64_t i = 0; i < n_pairs; ++i)
        if (!is_match[i]) {
            tp.push_back(pairs[2 * i]);
            tp.push_back(pairs[2 * i + 1]);
        }
    const uint64_t nt = tp.size() / 2;

    Model M;
    uint8_t *d_db = nullptr, *d_qb = nullptr, *d_sidx = nullptr;
    uint64_t *d_do = nullptr, *d_qo = nullptr, *d_dm = nullptr, *d_qm = nullptr, *d_ma = nullptr, *d_mb = nullptr;
    uint32_t *d_pairs = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        dfree(d_db);
        dfree(d_qb);
        dfree(d_sidx);
        dfree(d_do);
        dfree(d_qo);
        dfree(d_dm);
        dfree(d_qm);
        dfree(d_ma);
        dfree(d_mb);
        dfree(d_pairs);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        if (s)
            (void)hipStreamDestroy(s);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) || (e = hipEventCreate(&e0)) ||
        (e = hipEventCreate(&e1)) || (e = M.alloc(sh)) || (e = dalloc(&d_db, dn + 4)) ||
        (e = dalloc(&d_qb, qn + 4)) || (e = dalloc(&d_sidx, 256)) || (e = dalloc(&d_do, (size_t)n_words + 1)) ||
        (e = dalloc(&d_qo, (size_t)n_queries + 1)) || (e = dalloc(&d_dm, 2 * (size_t)n_words)) ||
        (e = dalloc(&d_qm, 2 * (size_t)n_queries)) || (e = dalloc(&d_ma, 2 * nt)) || (e = dalloc(&d_mb, 2 * nt)) ||
        (e = dalloc(&d_pairs, 2 * nt))) {
        cleanup();
        return hip_fail(e, "fpm_learn_grouping alloc");
    }
    if (dn)
        (void)hipMemcpyAsync(d_db, dbytes, dn, hipMemcpyHostToDevice, s);
    if (qn)
        (void)hipMemcpyAsync(d_qb, qbytes, qn, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(d_do, doffsets, sizeof(uint64_t) * ((size_t)n_words + 1), hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(d_qo, qoffsets, sizeof(uint64_t) * ((size_t)n_queries + 1), hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(d_sidx, sym_index, 256, hipMemcpyHostToDevice, s);
    if (nt)
        (void)hipMemcpyAsync(d_pairs, tp.data(), sizeof(uint32_t) * 2 * nt, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(M.X, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(M.params, params.data(), sizeof(float) * params.size(), hipMemcpyHostToDevice, s);
    launch_fill(M.m, sh.n_params(), s);
    launch_fill(M.v, sh.n_params(), s);
    if (n_words)
        hipLaunchKernelGGL(k_symbol_masks, dim3((n_words + 255) / 256), dim3(256), 0, s, d_db, d_do, n_words, d_sidx,
                           d_dm);
    if (n_queries)
        hipLaunchKernelGGL(k_symbol_masks, dim3((n_queries + 255) / 256), dim3(256), 0, s, d_qb, d_qo, n_queries,
                           d_sidx, d_qm);
    if (nt)
        hipLaunchKernelGGL(k_gather_pair_masks, dim3((uint32_t)((nt + 255) / 256)), dim3(256), 0, s, d_pairs, nt, d_qm,
                           d_dm, d_ma, d_mb);
    const float target = (float)(2 * cfg.k + 1) + cfg.margin;
    const uint64_t bsz = std::max<uint64_t>(1, std::min<uint64_t>(cfg.batch, std::max<uint64_t>(nt, 1)));
    const uint64_t nb = nt ? (nt + bsz - 1) / bsz : 1;
    uint32_t step = 0;
    float first_loss = 0.f, last_epoch_loss = 0.f, last_entropy = 0.f, last_e = 0.f;
    const float b1 = 0.9f, b2 = 0.999f;
    (void)hipEventRecord(e0, s);
    for (uint32_t ep = 0; ep < cfg.epochs; ++ep) {
        const float ew = cfg.entropy_weight * (cfg.epochs > 1 ? (float)ep / (float)(cfg.epochs - 1) : 1.f);
        double ep_loss = 0.0, ep_e = 0.0;
        for (uint64_t bi = 0; bi < nb; ++bi) {
            const uint64_t lo = bi * bsz, cntb = nt ? std::min<uint64_t>(bsz, nt - lo) : 0;
            e = forward_backward(M, d_ma + 2 * lo, d_mb + 2 * lo, cntb, target, cfg.beta, ew, s);
            if (e) {
                cleanup();
                return hip_fail(e, "training step");
            }
            ++step;
            const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
            hipLaunchKernelGGL(k_adam, dim3((sh.n_params() + 255) / 256), dim3(256), 0, s, M.params, M.grads, M.m,
                               M.v, sh.n_params(), cfg.lr, b1, b2, 1e-8f, c1, c2);
            if ((ep == 0 && bi == 0) || ep + 1 == cfg.epochs) {
                float sums[4];
                e = hipMemcpyAsync(sums, M.sums, sizeof(sums), hipMemcpyDeviceToHost, s);
                if (!e)
                    e = hipStreamSynchronize(s);
                if (e) {
                    cleanup();
                    return hip_fail(e, "training readback");
                }
                const float inv = cntb ? 1.f / (float)cntb : 0.f;
                if (ep == 0 && bi == 0)
                    first_loss = sums[0] * inv;
                if (ep + 1 == cfg.epochs) {
                    ep_loss += sums[0];
                    ep_e += sums[1];
                    last_entropy = sums[2];
                }
            }
        }
        if (ep + 1 == cfg.epochs && nt) {
            last_epoch_loss = (float)(ep_loss / (double)nt);
            last_e = (float)(ep_e / (double)nt);
        }
    }
    (void)hipEventRecord(e1, s);
    // final probabilities -> argmax map
    hipLaunchKernelGGL(k_mlp_forward, dim3(sh.sigma), dim3(128), 0, s, M.X, M.params, sh, M.pre, M.hid, M.P, M.L);
    std::vector<float> P((size_t)sh.sigma * (sh.bits + 1));
    e = hipMemcpyAsync(P.data(), M.P, sizeof(float) * P.size(), hipMemcpyDeviceToHost, s);
    if (!e)
        e = hipStreamSynchronize(s);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    cleanup();
    if (e)
        return hip_fail(e, "fpm_learn_grouping");
    memset(map_out, 0xFF, 256);
    for (uint32_t si = 0; si < sh.sigma; ++si) {
        uint32_t best = 0;
        for (uint32_t j = 1; j <= sh.bits; ++j)
            if (P[(size_t)si * (sh.bits + 1) + j] > P[(size_t)si * (sh.bits + 1) + best])
                best = j;
        map_out[syms[si]] = best == sh.bits ? 0xFF : (uint8_t)best;
    }
    if (report) {
        memset(report, 0, sizeof(*report));
        report->sigma = sh.sigma;
        report->d_in = sh.d_in;
        report->n_params = sh.n_params();
        report->steps = step;
        report->train_pairs = nt;
        report->first_loss = first_loss;
        report->final_loss = last_epoch_loss;
        report->final_entropy = last_entropy;
        report->expected_fd = last_e;
        report->ms = ms;
    }
    return FPM_OK;
}

}  // extern "C"
