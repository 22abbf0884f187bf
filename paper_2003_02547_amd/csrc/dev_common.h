// Device helpers shared by the IPM kernels: wave-level reductions and
// broadcasts, FP64 reciprocal and reciprocal square root refined from the
// hardware estimates, and the right-hand-side modes of the sweeps.
#pragma once

#include <hip/hip_runtime.h>

namespace oqp {

constexpr int WAVE = 64;

__host__ __device__ constexpr int ru8(int v) { return (v + 7) / 8 * 8; }
__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Ordering point for LDS traffic exchanged inside one wave: the LDS
// operations of a wave execute in order, so a compiler-level barrier is all
// that is needed.
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double nmax(double a, double b) { return (a > b || a != a) ? a : b; }

// xor-butterfly reductions: every lane ends with the same bits (each step
// combines two equal-valued halves with a commutative operation)
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Value of v held by lane `src` (src is wave-uniform).
__device__ __forceinline__ double bcast(double v, int src)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1/sqrt(x) to double precision: hardware estimate and one Newton step.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x * y;
    return y * (1.5 - h * y);
}

// 1/x to double precision: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    return y * (2.0 - x * y);
}

// Right-hand-side variants of the complementarity row r_m.
enum { RM_SHIFT = 0,      // r_m = lam.*t - shift
       RM_CORRECTOR = 1,  // r_m = lam.*t + dlam_aff.*dt_aff - shift
       RM_IR = 2 };       // r_m taken from the refinement residual arrays

}  // namespace oqp
