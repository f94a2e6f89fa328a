// Device-side helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nlch_internal.h"

namespace nlch {

typedef _Float16 half_t;

// Storage <-> arithmetic conversions; narrowing is round-to-nearest-even.
template <class TA, class TS>
__device__ __forceinline__ TA to_acc(TS v) {
    return static_cast<TA>(v);
}
template <class TS, class TA>
__device__ __forceinline__ TS to_store(TA v) {
    return static_cast<TS>(v);
}

// Projection onto [-1, 1] written with comparisons so that a NaN passes
// through (fmin/fmax would silently turn it into a bound).
template <class T>
__device__ __forceinline__ T clamp1(T v) {
    return v < T(-1) ? T(-1) : (v > T(1) ? T(1) : v);
}
// FP32: IEEE 754-2019 maximum/minimum propagate NaN and map to one
// v_maximum3_f32 and one v_minimum3_f32 on gfx950.
template <>
__device__ __forceinline__ float clamp1<float>(float v) {
    return __builtin_elementwise_minimum(__builtin_elementwise_maximum(v, -1.0f), 1.0f);
}

// Update coefficients in the arithmetic type.
template <class TA>
__device__ __forceinline__ TA coef_a(const SampleDesc &d);
template <>
__device__ __forceinline__ float coef_a<float>(const SampleDesc &d) { return d.af; }
template <>
__device__ __forceinline__ double coef_a<double>(const SampleDesc &d) { return d.a; }
template <class TA>
__device__ __forceinline__ TA coef_b(const SampleDesc &d);
template <>
__device__ __forceinline__ float coef_b<float>(const SampleDesc &d) { return d.bf; }
template <>
__device__ __forceinline__ double coef_b<double>(const SampleDesc &d) { return d.b; }

template <class TA>
__device__ __forceinline__ TA geo_g(const ModelGeo *g, int k);
template <>
__device__ __forceinline__ float geo_g<float>(const ModelGeo *g, int k) { return g->gf[k]; }
template <>
__device__ __forceinline__ double geo_g<double>(const ModelGeo *g, int k) { return g->gd[k]; }

template <class TA>
__device__ __forceinline__ TA geo_ce(const ModelGeo *g);
template <>
__device__ __forceinline__ float geo_ce<float>(const ModelGeo *g) { return g->cef; }
template <>
__device__ __forceinline__ double geo_ce<double>(const ModelGeo *g) { return g->ced; }

// Fused multiply-add a b + c (one rounding).  The stencil units are
// compiled without automatic contraction, so every fused operation of the
// path is written out here and every kernel rounds the same operations the
// same way (results do not depend on how a kernel's code was scheduled).
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double madd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Lsum = ce u - G (unit-amplitude operator sum from the disc sum G).
template <class TA>
__device__ __forceinline__ TA lsum_of(TA ce, TA u, TA G) {
    return madd(ce, u, -G);
}

// v = u + (a u - b Lsum), projected.  Sign-symmetric: update(-u, -Lsum) is
// -update(u, Lsum) exactly.  (The per-site direct kernel, which forms Lsum
// itself.)
template <class TA>
__device__ __forceinline__ TA update(TA u, TA lsum, TA a, TA b) {
    const TA t = madd(-b, lsum, a * u);
    return clamp1(u + t);
}

// The same update from the disc sum G (Lsum = ce u - G):
//   a u - b Lsum = (a - b ce) u + b G = ap u + b G,  ap = c1 (c_F - c_gamma_h),
// one fused multiply-add on the small term ap u (5 lane operations with the
// projection instead of 6).  Sign-symmetric, and u = +-1, 0 stay fixed
// exactly (for u = 1 the increment rounds to about a = c1 c_F > 0).
template <class TA>
__device__ __forceinline__ TA update_g(TA u, TA G, TA ap, TA b) {
    const TA t = madd(b, G, ap * u);
    return clamp1(u + t);
}

template <class TA>
__device__ __forceinline__ TA coef_ap(const SampleDesc &d);
template <>
__device__ __forceinline__ float coef_ap<float>(const SampleDesc &d) { return d.apf; }
template <>
__device__ __forceinline__ double coef_ap<double>(const SampleDesc &d) { return d.ap; }

// Periodic index for |i| < 2n.
__device__ __forceinline__ int wrap_once(int i, int n) {
    i += (i < 0) ? n : 0;
    i -= (i >= n) ? n : 0;
    return i;
}

// Map a linear work index so that each of the 8 XCDs (which receive
// workgroups round-robin) works on a contiguous range of tiles: neighbouring
// tiles share halo rows, and each XCD has its own L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    constexpr int kXcd = 8;
    int per = nblocks / kXcd;
    if (per == 0 || b >= per * kXcd) return b;
    return (b % kXcd) * per + b / kXcd;
}

// Deterministic block-wide FP64 sum (fixed shuffle tree, then waves in
// order).  `red` is a __shared__ scratch of at least blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

}  // namespace nlch
