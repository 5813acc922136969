// Device-side helpers shared by the library's kernels (gfx950, wave64).
// Internal to the GPU library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HK_WAVE 64

namespace hk {

// 2^y for a float64 argument y (|y| up to a few hundred), returned in
// float32: y = k + r with k = rint(y) and r = y - k (exact in float64), 2^r
// from the hardware exp2, k applied with ldexp (far below float32 range: 0).
// Callers fold log2(e) into the rate, so that e^{b x} costs one float64
// multiply before this; relative error a few float32 ulp.
__device__ __forceinline__ float exp2_f64arg(double y) {
    const double k = __builtin_rint(y);
    const float e = __builtin_amdgcn_exp2f((float)(y - k));
    int ki = (int)k;
    ki = ki < -300 ? -300 : ki;
    return __builtin_ldexpf(e, ki);
}
#define HK_LOG2E 1.4426950408889634

// e^x in float64 for x <= 0 (the decays of the forward passes).  Cody-Waite
// reduction x = k ln2 + r with |r| <= ln2/2 (ln2 split in two parts), then
// the Taylor series of e^r through r^12 / 12! by Horner's rule (truncation
// below 2e-16 relative for |r| <= ln2/2), scaled by 2^k.  Below -708 the
// result is 0 (float64 underflow).
__device__ __forceinline__ double exp_f64(double x) {
    const double kLog2e = 1.4426950408889634;
    const double kLn2Hi = 6.93147180369123816490e-01;
    const double kLn2Lo = 1.90821492927058770002e-10;
    const double k = __builtin_rint(x * kLog2e);
    double r = __builtin_fma(-k, kLn2Hi, x);
    r = __builtin_fma(-k, kLn2Lo, r);
    double p = 1.0 / 479001600.0;             // 1/12!
    p = __builtin_fma(p, r, 1.0 / 39916800.0);  // 1/11!
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    const double v = __builtin_ldexp(p, (int)k);
    return x < -708.0 ? 0.0 : v;
}

// wave-uniform value from lane 0
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double shfl_d(double v, int src) {
    return __shfl(v, src, HK_WAVE);
}
__device__ __forceinline__ double shfl_up_d(double v, int d) {
    return __shfl_up(v, d, HK_WAVE);
}

// Waits for this wave's outstanding LDS operations (lgkmcnt(0)); the
// compiler fences keep LDS accesses from moving across it.  Needed where a
// wave reads back what it has just written with LDS atomics: a read can
// complete ahead of the same wave's earlier return-less LDS atomic.
__device__ __forceinline__ void lds_wait() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int clamp_mark(int m, int M) {
    return m < 0 ? 0 : (m >= M ? M - 1 : m);
}

// deterministic block-wide float64 sum (fixed tree), blockDim.x == NT
template <int NT>
__device__ double block_sum_d(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

}  // namespace hk
