// Compositing arithmetic shared by the forward blend and its backward: the
// staged form of a screen record and the footprint exponent, written with
// explicit fused multiply-adds so that both kernels make the same decisions
// and compute the same transmittance, bit for bit.
#pragma once

#include "internal.h"

namespace gsr {

constexpr float kLog2e = 1.4426950408889634f;

struct BlendConsts {
    float cull_r2;          // cutoff with a margin, for the (band, quarter) overlap test
    float sqrt_half_log2e;  // sqrt(log2(e)/2): scales the conic factors
    float cut_p2;           // -log2(e)/2 * cutoff_d2
    float log2_amin;        // log2(alpha_min)
    float alpha_max;
    float t_min;
};

inline BlendConsts blend_consts(const Consts &k) {
    BlendConsts bc;
    bc.cull_r2 = k.cutoff_d2 * 1.001f + 1e-3f;
    bc.sqrt_half_log2e = sqrtf(0.5f * kLog2e);
    bc.cut_p2 = -0.5f * kLog2e * k.cutoff_d2;
    bc.log2_amin = log2f(k.alpha_min);
    bc.alpha_max = k.alpha_max;
    bc.t_min = k.t_min;
    return bc;
}

// det of the conic [[A, B], [B, C]]: products of floats are exact in double, so
// det keeps its accuracy for thin, tilted ellipses where A C and B^2 nearly cancel
__device__ __forceinline__ float conic_det(float A, float B, float C) {
    return (float)((double)A * (double)C - (double)B * (double)B);
}

// Max and min of two finite floats in one instruction: the median with an
// infinite third operand (fmaxf and fminf also quiet signalling NaNs, which
// costs an extra instruction per operand that is not known to be canonical).
__device__ __forceinline__ float max_finite(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, __builtin_inff());
}
__device__ __forceinline__ float min_finite(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, -__builtin_inff());
}

// Staged record of screen record (q0, q1, q2) (see internal.h) for the tile whose
// centre is (xc, yc), with (uc, vc) = (u - xc, v - yc) the footprint's centre
// relative to it:
//   s0 = (k1, k2, m11', m12'), s1 = (m22', threshold, log2 o, z), s2 = (r, g, b, vc)
// with d^2 = (m11 dx + m12 dy)^2 + (m22 dy)^2, m11 = sqrt(A), m12 = B / m11,
// m22 = sqrt(det / A), each scaled by sqrt(log2(e)/2) ('); the exponent of
// o exp(-d^2/2) in base 2 is then log2(o) - t1^2 - t2^2, and a pair contributes
// when it is >= threshold = max(log2(o) - log2(e) cutoff / 2, log2(alpha_min)).
// With the pixel centre (x, y) taken relative to the tile centre as well, t1 and
// t2 are affine in it: t1 = m11' x + m12' y + k1, t2 = m22' y + k2, where
// k1 = -(m11' uc + m12' vc) and k2 = -m22' vc (three fused multiply-adds per
// pixel instead of two differences and three products). Every term is at most
// the footprint's extent plus half a tile in pixels, so the rounding of t1^2 + t2^2
// stays within about 1e-5 (in log2 of alpha) of the exact value, inside the
// float32 margins of the contribution tests.
// The factors come from the hardware reciprocal square root and square root
// (about 1 ulp each), far inside the same margins.
__device__ __forceinline__ void stage_record(const float4 &q0, const float4 &q1, const float4 &q2, float det,
                                             float uc, float vc, const BlendConsts &k, float4 &s0, float4 &s1,
                                             float4 &s2) {
    const float A = q0.z, B = q0.w;
    const float r = __builtin_amdgcn_rsqf(A);  // 1 / sqrt(A)
    const float m11 = A * r;
    const float m12 = B * r;
    const float m22 = __builtin_amdgcn_sqrtf(max_finite(det, 0.f)) * r;  // 0: the limit of a degenerate streak
    const float lo = __log2f(q1.y);
    const float thr = fmaxf(k.cut_p2 + lo, k.log2_amin);
    const float a11 = m11 * k.sqrt_half_log2e, a12 = m12 * k.sqrt_half_log2e, a22 = m22 * k.sqrt_half_log2e;
    s0 = make_float4(-__builtin_fmaf(a11, uc, a12 * vc), -(a22 * vc), a11, a12);
    s1 = make_float4(a22, thr, lo, q2.y);
    s2 = make_float4(q1.z, q1.w, q2.x, vc);
}

// min(alpha_max, e) for e >= 0 (an exponential) in one instruction: the median
// of (e, 0, alpha_max) equals it for every such e, bit for bit.
__device__ __forceinline__ float clamp_alpha(float e, float alpha_max) {
    return __builtin_amdgcn_fmed3f(e, 0.f, alpha_max);
}

// Base-2 exponent of the footprint of staged record (s0, s1) at the pixel centre
// (x, y), relative to the tile centre.
__device__ __forceinline__ float footprint_p2(const float4 &s0, const float4 &s1, float x, float y) {
    const float t1 = __builtin_fmaf(s0.z, x, __builtin_fmaf(s0.w, y, s0.x));
    const float t2 = __builtin_fmaf(s1.x, y, s0.y);
    return __builtin_fmaf(-t2, t2, __builtin_fmaf(-t1, t1, s1.z));
}

}  // namespace gsr
