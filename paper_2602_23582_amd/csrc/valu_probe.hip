// Issue-rate probe for the roofline of the ALU-bound kernels: how many wave
// instructions per cycle one SIMD issues for FP32 FMA, for the transcendental
// instructions the kernels use (v_exp_f32, v_rsq_f32, v_sin_f32) and for mixes
// of the two.  Every lane runs kChains independent dependency chains so that
// issue rate, not latency, is measured.  Not part of the RBSOG library.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;

// kind: 0 FMA; 1 exp; 2 rsq; 3 sin; 4 one exp per 4 FMA; 5 one exp per 2 FMA;
// 6 one exp per FMA; 7 one exp per 8 FMA
template <int kind>
__global__ __launch_bounds__(256) void k_probe(int iters, float *out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float a[kChains], b[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = 0.25f + 1e-3f * (t & 63) + 0.01f * c;
        b[c] = 0.5f + 1e-3f * c;
    }
    const float m = 0.999f, k = 1e-3f;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
        if constexpr (kind == 0) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_fmaf(a[c], m, k);
        } else if constexpr (kind == 1) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);
        } else if constexpr (kind == 2) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_rsqf(a[c]);
        } else if constexpr (kind == 3) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_sinf(a[c]);
        } else {
            constexpr int per = kind == 4 ? 4 : kind == 5 ? 2 : kind == 6 ? 1 : 8;
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);
#pragma unroll
            for (int r = 0; r < per; ++r) {
#pragma unroll
                for (int c = 0; c < kChains; ++c) b[c] = __builtin_fmaf(b[c], m, k);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c] + b[c];
    out[t] = s;
}

}  // namespace

extern "C" {

// Runs the probe on `blocks` workgroups of 256 threads (out must hold
// 256 * blocks floats, device memory) and returns the kernel time in
// milliseconds through *ms.  Returns 0 on success, a hipError_t otherwise.
int valu_probe(int kind, int iters, int blocks, float *out, float *ms)
{
    if (kind < 0 || kind > 7 || iters < 1 || blocks < 1 || !out || !ms) return -1;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) return e;
    using Fn = void (*)(int, float *);
    const Fn fns[8] = {k_probe<0>, k_probe<1>, k_probe<2>, k_probe<3>,
                       k_probe<4>, k_probe<5>, k_probe<6>, k_probe<7>};
    hipLaunchKernelGGL(fns[kind], dim3(blocks), dim3(256), 0, nullptr, 1, out);  // warm-up
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(fns[kind], dim3(blocks), dim3(256), 0, nullptr, iters, out);
    (void)hipEventRecord(e1, nullptr);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

}  // extern "C"
