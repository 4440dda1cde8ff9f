// Ray and sample arithmetic shared by the projector and its transpose.
//
// Both kernels must agree on which interpolation cell every sample falls
// in, so the sample coordinate is produced by one function, with floating
// point contraction disabled and explicit fused multiply-adds, and the cell
// is always floor() of that coordinate.  Then the gather-form transpose
// enumerates exactly the (ray, sample) pairs the projector visits.
//
// Sample coordinates are computed in double precision whatever the data
// type: a sample about 1000 mm from the source needs its direction to
// ~1e-9 relative to land within 1e-5 voxel of its true position, beyond
// float's 24-bit mantissa.  Double FMA, floor and convert run at the same
// vector rate as non-packed float on gfx950.  The float variant of
// ray_setup only feeds conservative range estimates.
#pragma once

#include "cbct_internal.hpp"

namespace cbct {

// Index-space origin Q and per-sample increment D of the ray through
// pixel (i, j) of view vc (see ViewConst).
__device__ __forceinline__ void ray_setup(const ViewConst &vc, const DetConst &dc, int i, int j,
                                          float Q[3], float D[3]) {
#pragma clang fp contract(off)
    const float u = __builtin_fmaf((float)i, dc.au, dc.u0);
    const float v = __builtin_fmaf((float)j, dc.av, dc.v0);
    const float l2 = __builtin_fmaf(u, u, __builtin_fmaf(v, v, dc.sdd2));
    const float inv = __builtin_amdgcn_rsqf(l2);
    D[0] = __builtin_fmaf(u, vc.U[0], vc.W[0]) * inv;
    D[1] = __builtin_fmaf(u, vc.U[1], vc.W[1]) * inv;
    D[2] = (v * vc.Vz) * inv;
    Q[0] = vc.Q[0];
    Q[1] = vc.Q[1];
    Q[2] = vc.Q[2];
}

__device__ __forceinline__ void ray_setup(const ViewConst &vc, const DetConst &dc, int i, int j,
                                          double Q[3], double D[3]) {
#pragma clang fp contract(off)
    const double u = __builtin_fma((double)i, dc.aud, dc.u0d);
    const double v = __builtin_fma((double)j, dc.avd, dc.v0d);
    const double l2 = __builtin_fma(u, u, __builtin_fma(v, v, dc.sdd2d));
    const double inv = 1.0 / __builtin_sqrt(l2);
    D[0] = __builtin_fma(u, vc.Ud[0], vc.Wd[0]) * inv;
    D[1] = __builtin_fma(u, vc.Ud[1], vc.Wd[1]) * inv;
    D[2] = (v * vc.Vzd) * inv;
    Q[0] = vc.Qd[0];
    Q[1] = vc.Qd[1];
    Q[2] = vc.Qd[2];
}

// ---------------------------------------------------------------------------
// Sample cells and trilinear weights.
//
// Float data (the production path): the samples of a ray are grouped in
// segments of SEG consecutive indices n (a global lattice, n_s = n & ~(SEG-1),
// independent of where the ray enters the grid).  The segment origin
// q(n_s) = Q + n_s D is evaluated in double and split into an integer cell
// I and a float fraction f in [0, 1]; inside the segment
//     l = fma(m, D_f, f),   m = n - n_s in [0, SEG),  D_f = (float)D,
// cell = I + floor(l), weight = l - floor(l).  With the default step
// (|D_a| <= 1/2) |l| stays below SEG/2 + 1 = 129, so float keeps the
// position to ~1.5e-5 voxel (one rounding of l plus the rounding of D_f
// over 256 steps), and the double work is paid once per segment.  Long
// segments matter to the transpose: the samples of one ray inside one
// brick of cells (at most ~33 of them) nearly always share a segment,
// whose origin can then be prepared once per pixel and brick.
//
// Double data (derivative checks): q = fma(n, D, Q) in double per sample.
constexpr int SEG = 256;

struct SegOrigin {
    int I[3];
    float f[3];
};

__device__ __forceinline__ SegOrigin seg_origin(const double Q[3], const double D[3], int ns) {
#pragma clang fp contract(off)
    SegOrigin o;
    const double nd = (double)ns;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = __builtin_fma(nd, D[a], Q[a]);
        const double fl = __builtin_floor(q);
        o.I[a] = (int)fl;
        o.f[a] = (float)(q - fl);
    }
    return o;
}

// Cell offset (relative to the segment's integer origin) and weight along
// one axis for in-segment index m.
__device__ __forceinline__ void seg_axis(float m, float Df, float f, int &dc, float &w) {
#pragma clang fp contract(off)
    const float l = __builtin_fmaf(m, Df, f);
    const float fl = __builtin_floorf(l);
    dc = (int)fl;
    w = l - fl;
}

__device__ __forceinline__ void to_float3(const double D[3], float Df[3]) {
    Df[0] = (float)D[0];
    Df[1] = (float)D[1];
    Df[2] = (float)D[2];
}

// Voxel-index coordinate of sample n along one axis.
__device__ __forceinline__ float sample_coord(float n, float D, float Q) {
    return __builtin_fmaf(n, D, Q);
}
__device__ __forceinline__ double sample_coord(double n, double D, double Q) {
    return __builtin_fma(n, D, Q);
}

template <typename T>
__device__ __forceinline__ T floor_t(T x);
template <>
__device__ __forceinline__ float floor_t<float>(float x) { return __builtin_floorf(x); }
template <>
__device__ __forceinline__ double floor_t<double>(double x) { return __builtin_floor(x); }

// Interval [lo, hi] (real-valued, unrounded) of sample indices whose
// coordinate along one axis lies in [a, b); returns false if none can.
template <typename T>
__device__ __forceinline__ bool axis_interval(T Q, T D, T a, T b, T &lo, T &hi) {
    if (D > T(0)) {
        T inv = T(1) / D;
        lo = (a - Q) * inv;
        hi = (b - Q) * inv;
        return true;
    }
    if (D < T(0)) {
        T inv = T(1) / D;
        lo = (b - Q) * inv;
        hi = (a - Q) * inv;
        return true;
    }
    lo = T(-1e30);
    hi = T(1e30);
    return Q >= a && Q < b;
}

// Conservative float estimate of the sample indices whose coordinate along
// one axis lies in [a, a + 1), for a ray given in float (Q, D).  The float
// ray differs from the double one by at most ~1e-6 relative in Q and D, so
// the true bounds (a - Q)/D move by at most 1e-6 (|Q| + |a| + 1) / |D|;
// the interval is widened by four times that plus 1e-3.  Returns false
// when no sample can have that coordinate.
__device__ __forceinline__ bool axis_estimate(float Q, float D, float a, float &lo, float &hi) {
    if (D == 0.0f) {
        lo = -1e30f;
        hi = 1e30f;
        // q = Q exactly for every n in double too (D is exactly zero there
        // only when the double D is zero as well: both come from u = 0 or
        // v = 0 for the same pixel)
        return Q >= a - 1e-3f && Q < a + 1.0f + 1e-3f;
    }
    const float inv = __builtin_amdgcn_rcpf(D);
    const float m = 1e-3f + 4e-6f * (fabsf(Q) + fabsf(a) + 1.0f) * fabsf(inv);
    const float t0 = (a - Q) * inv, t1 = (a + 1.0f - Q) * inv;
    lo = fminf(t0, t1) - m;
    hi = fmaxf(t0, t1) + m;
    return true;
}

// Clamp a real sample index into a range safe for int conversion.
template <typename T>
__device__ __forceinline__ int clamp_to_int(T x) {
    x = x < T(-4) ? T(-4) : x;
    x = x > T(1 << 24) ? T(1 << 24) : x;
    return (int)x;
}

// Same for float with one median-of-three (finite inputs).
template <>
__device__ __forceinline__ int clamp_to_int<float>(float x) {
    return (int)__builtin_amdgcn_fmed3f(x, -4.0f, (float)(1 << 24));
}

}  // namespace cbct
