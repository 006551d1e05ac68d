// Diagnostic microbenchmarks behind the measurement notes: the VALU issue rate of plain
// float multiply-add chains at one or more waves per SIMD, and the cost of a launch that does
// nothing. Used by no device path.
#include <hip/hip_runtime.h>

#include "mgx.h"
#include "runtime_internal.hpp"

namespace mgx {

// Each lane runs `chains` independent multiply-add chains of 16 * iters links (float,
// no packed math), then stores their sum.
template <int kChains>
__global__ void __launch_bounds__(256) k_valu_probe(float* out, int64_t n, int iters, float a, float b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (float)(i & 255) * 1e-3f + (float)c;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[i] = s;
}

__global__ void k_empty_probe(int32_t* flag) {
    if (flag[0] == 12345 && threadIdx.x == 0) flag[1] = 1;  // never true: the host writes 0
}

}  // namespace mgx

using namespace mgx;

extern "C" mgx_status mgx_diag_valu_probe(int32_t chains, int64_t n_threads, int32_t iters, double* seconds) {
    if (!seconds) return fail(MGX_E_INVALID, "seconds is NULL");
    if (chains != 1 && chains != 2 && chains != 4 && chains != 8) return fail(MGX_E_INVALID, "chains in {1, 2, 4, 8}");
    if (n_threads < 64 || n_threads > ((int64_t)1 << 24) || n_threads % 256)
        return fail(MGX_E_INVALID, "n_threads a multiple of 256 in [256, 2^24]");
    if (iters < 1 || iters > (1 << 20)) return fail(MGX_E_INVALID, "iters in [1, 2^20]");
    float* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, sizeof(float) * n_threads);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    const unsigned grid = (unsigned)(n_threads / 256);
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // the first launch warms up
        e = hipEventRecord(e0, nullptr);
        switch (chains) {
            case 1: hipLaunchKernelGGL(k_valu_probe<1>, dim3(grid), dim3(256), 0, nullptr, out, n_threads, iters, 0.999f, 1e-3f); break;
            case 2: hipLaunchKernelGGL(k_valu_probe<2>, dim3(grid), dim3(256), 0, nullptr, out, n_threads, iters, 0.999f, 1e-3f); break;
            case 4: hipLaunchKernelGGL(k_valu_probe<4>, dim3(grid), dim3(256), 0, nullptr, out, n_threads, iters, 0.999f, 1e-3f); break;
            default: hipLaunchKernelGGL(k_valu_probe<8>, dim3(grid), dim3(256), 0, nullptr, out, n_threads, iters, 0.999f, 1e-3f); break;
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && ms < best) best = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return fail(MGX_E_DEVICE, "valu probe: %s", hipGetErrorString(e));
    *seconds = best * 1e-3;
    return MGX_OK;
}

extern "C" mgx_status mgx_diag_launch_floor(int64_t n_threads, int32_t block, int32_t launches, double* seconds) {
    if (!seconds) return fail(MGX_E_INVALID, "seconds is NULL");
    if (block != 64 && block != 128 && block != 256) return fail(MGX_E_INVALID, "block in {64, 128, 256}");
    if (n_threads < block || n_threads > ((int64_t)1 << 24) || n_threads % block)
        return fail(MGX_E_INVALID, "n_threads a multiple of block in [block, 2^24]");
    if (launches < 1 || launches > 100000) return fail(MGX_E_INVALID, "launches in [1, 100000]");
    int32_t* flag = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&flag, 2 * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(flag, 0, 2 * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    const unsigned grid = (unsigned)(n_threads / block);
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, nullptr);
        for (int k = 0; k < launches && e == hipSuccess; ++k) {
            hipLaunchKernelGGL(k_empty_probe, dim3(grid), dim3(block), 0, nullptr, flag);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && ms < best) best = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (flag) (void)hipFree(flag);
    if (e != hipSuccess) return fail(MGX_E_DEVICE, "launch floor: %s", hipGetErrorString(e));
    *seconds = best * 1e-3 / launches;
    return MGX_OK;
}
