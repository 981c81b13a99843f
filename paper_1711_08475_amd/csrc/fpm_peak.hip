// fpm_peak.hip -- peak-rate probes of the 32-bit integer vector ALUs (the
// vector filter's instruction mix) and of the int8 matrix cores
// (v_mfma_i32_32x32x32_i8), behind fpm_measure_peaks (fpm_peak.h).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/fpm_peak.h"
#include "fpm_host.hpp"

using namespace fpm;

namespace {

constexpr int kBlocksPerCu = 8;  // 8 blocks x 4 waves: 8 waves per SIMD
constexpr int kThreads = 256;
constexpr uint32_t kValuIters = 8192;
constexpr uint32_t kMatrixIters = 16384;
constexpr uint64_t kValuOpsPerIter = 16 * 2 * 3;  // 16 uniform values x 2 lane values x 3 instructions
constexpr uint64_t kMatrixOpsPerMfma = 2ull * 32 * 32 * 32;

struct Uniform16 {
    uint32_t q[16];
};

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

// Per lane two values against 16 uniform ones: v_xor_b32, v_bcnt_u32_b32
// (accumulating the bias), v_alignbit_b32 per pair.  The empty asm keeps
// the lane values "changed" every iteration, so nothing is hoisted.
__global__ void __launch_bounds__(kThreads) k_valu_peak(Uniform16 u, uint32_t neg, uint32_t iters, uint32_t *out)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t w0 = gid * 0x9E3779B9u, w1 = gid ^ 0x85EBCA6Bu, m0 = 0, m1 = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        asm volatile("" : "+v"(w0), "+v"(w1));
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            m0 = __builtin_amdgcn_alignbit(m0, (uint32_t)__builtin_popcount(u.q[s] ^ w0) + neg, 31);
            m1 = __builtin_amdgcn_alignbit(m1, (uint32_t)__builtin_popcount(u.q[s] ^ w1) + neg, 31);
        }
    }
    out[gid] = m0 ^ m1;
}

// Two independent accumulator chains of v_mfma_i32_32x32x32_i8 per wave.
__global__ void __launch_bounds__(kThreads) k_matrix_peak(int seed, uint32_t iters, int *out)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const v4i_t a = {seed ^ (int)gid, seed + (int)gid, seed * 3, (int)gid};
    const v4i_t b = {(int)gid * 7, seed, seed ^ 0x55, (int)gid + 1};
    v16i_t d0 = (v16i_t)(0), d1 = (v16i_t)(0);
    for (uint32_t it = 0; it < iters; ++it) {
        d0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, d1, 0, 0, 0);
    }
    int r = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        r ^= d0[i] + d1[i];
    out[gid] = r;
}

// One warm-up and one timed launch; returns the timed duration (ms).
template <typename Launch>
fpm_status timed(hipStream_t s, hipEvent_t e0, hipEvent_t e1, Launch launch, float *ms)
{
    launch();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(e0, s));
    launch();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return FPM_OK;
}

}  // namespace

extern "C" fpm_status fpm_measure_peaks(fpm_peaks *out)
{
    g_last_error.clear();
    if (!out)
        return fail(FPM_EINVAL, "null out");
    memset(out, 0, sizeof(*out));
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus <= 0)
        return fail(FPM_EDEVICE, "no compute units reported");
    const uint32_t blocks = (uint32_t)cus * kBlocksPerCu;
    const size_t threads = (size_t)blocks * kThreads;
    uint32_t *buf = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fpm_status st = FPM_OK;
    hipError_t e;
    if ((e = dalloc(&buf, threads)) || (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) ||
        (e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1))) {
        st = hip_fail(e, "peak probe setup");
    }
    float vms = 0.f, mms = 0.f;
    if (!st) {
        Uniform16 u;
        for (int i = 0; i < 16; ++i)
            u.q[i] = 0x01234567u * (uint32_t)(i + 1);
        st = timed(s, e0, e1, [&] {
            hipLaunchKernelGGL(k_valu_peak, dim3(blocks), dim3(kThreads), 0, s, u, 0u - 3u, kValuIters, buf);
        }, &vms);
    }
    if (!st)
        st = timed(s, e0, e1, [&] {
            hipLaunchKernelGGL(k_matrix_peak, dim3(blocks), dim3(kThreads), 0, s, 12345, kMatrixIters, (int *)buf);
        }, &mms);
    if (!st) {
        const uint64_t waves = (uint64_t)blocks * (kThreads / 64);
        out->valu_ops = (uint64_t)threads * kValuIters * kValuOpsPerIter;
        out->matrix_ops = waves * 2ull * kMatrixIters * kMatrixOpsPerMfma;
        out->valu_ms = vms;
        out->matrix_ms = mms;
        out->int_valu_ops_per_s = vms > 0.f ? (double)out->valu_ops / (vms * 1e-3) : 0.0;
        out->int8_matrix_ops_per_s = mms > 0.f ? (double)out->matrix_ops / (mms * 1e-3) : 0.0;
        out->compute_units = (uint32_t)cus;
    }
    if (s)
        (void)hipStreamSynchronize(s);  // nothing in flight reads buf when it is freed
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (s)
        (void)hipStreamDestroy(s);
    dfree(buf);
    return st;
}
