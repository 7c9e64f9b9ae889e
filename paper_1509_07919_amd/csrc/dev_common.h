// Small device helpers shared by the HIP translation units of libsap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sap {

// value of lane l of a wave (l uniform), via v_readlane
__device__ __forceinline__ double lane_bcast(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// 1/p: the hardware reciprocal estimate refined by Newton-Raphson steps
// r <- r + r (1 - p r), each of which squares the relative error (two for
// FP64, one for FP32, reaching the format's precision to within an ulp).
// 0 maps to inf, then NaN; callers flag zero pivots themselves.
__device__ __forceinline__ double fast_recip(double p)
{
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float fast_recip(float p)
{
    const float r = __builtin_amdgcn_rcpf(p);
    const float e = fmaf(-p, r, 1.0f);
    return fmaf(r, e, r);
}

// Entry (r, c) of diagonal block [s0, s0+nb) in band storage (band[q*n + c]
// holds a(c+q-K, c)); ul != 0 reads the block with rows and columns reversed
// (J A_i J).  Zero outside the block or the band.
__device__ __forceinline__ double block_entry(const double *__restrict__ band, int64_t n,
                                              int k, int64_t s0, int64_t nb, int ul,
                                              int64_t r, int64_t c)
{
    const int64_t d = r - c;
    if (r < 0 || c < 0 || r >= nb || c >= nb || d > k || d < -k) return 0.0;
    const int64_t q = ul ? (k - d) : (k + d);
    const int64_t col = ul ? (s0 + nb - 1 - c) : (s0 + c);
    return band[q * n + col];
}

}  // namespace sap
