// Transpose of the projector, P^T, in gather form without atomics.
//
// The paper computes the gradient of E2 per voxel by a gather (Eq. (2)) to
// avoid the write conflicts of the scattering matrix transpose.  Here the
// gather is the EXACT transpose of the discrete projector, organised by
// interpolation cell rather than by voxel:
//
//   * a cell c = (cx, cy, cz), c_a in [-1, N_a - 1], is the box between
//     voxel centres c and c + 1; every projector sample lies in exactly one
//     cell, the one given by floor() of its coordinate;
//   * pass 1 (one lane per cell): for every view, project the cell box on
//     the detector, visit the pixels whose rays can cross it, enumerate the
//     samples of each such ray that fall in the cell (same arithmetic as the
//     projector), and accumulate r * (trilinear corner weight) into eight
//     register accumulators, one per cell corner;
//   * pass 2 (one lane per voxel): sum the matching corner of the eight
//     cells that share the voxel, optionally fused with Step 1 of
//     Algorithm A1, g = f - tau * P^T r.
//
// Each (ray, sample) is visited once instead of eight times (once per
// trilinear tap), every sum has a fixed order, and no lane writes memory
// another lane writes.
#include "ray.hpp"

namespace cbct {

namespace {

constexpr int CELL_BX = 64;
constexpr int CELL_BY = 4;

// Detector-coordinate bounds of the projection of an axis-aligned box
// [xa, xb] x [ya, yb] x [za, zb] (mm) for view vc; the extremes of the
// perspective map over a box are taken at its corners.
__device__ __forceinline__ void box_footprint(const ViewConst &vc, float sdd, float xa, float xb,
                                              float ya, float yb, float za, float zb,
                                              float &umin, float &umax, float &vmin,
                                              float &vmax) {
    const float wx0 = xa - vc.src[0], wx1 = xb - vc.src[0];
    const float wy0 = ya - vc.src[1], wy1 = yb - vc.src[1];
    // numerator of u (w . e_u) and depth (w . e_w) at the four xy corners
    const float n00 = wx0 * vc.cs + wy0 * vc.sn, d00 = wy0 * vc.cs - wx0 * vc.sn;
    const float n10 = wx1 * vc.cs + wy0 * vc.sn, d10 = wy0 * vc.cs - wx1 * vc.sn;
    const float n01 = wx0 * vc.cs + wy1 * vc.sn, d01 = wy1 * vc.cs - wx0 * vc.sn;
    const float n11 = wx1 * vc.cs + wy1 * vc.sn, d11 = wy1 * vc.cs - wx1 * vc.sn;
    const float u00 = n00 / d00, u10 = n10 / d10, u01 = n01 / d01, u11 = n11 / d11;
    umin = sdd * fminf(fminf(u00, u10), fminf(u01, u11));
    umax = sdd * fmaxf(fmaxf(u00, u10), fmaxf(u01, u11));
    const float dmin = fminf(fminf(d00, d10), fminf(d01, d11));
    const float dmax = fmaxf(fmaxf(d00, d10), fmaxf(d01, d11));
    const float ia = 1.0f / dmin, ib = 1.0f / dmax;
    const float v0 = za * ia, v1 = za * ib, v2 = zb * ia, v3 = zb * ib;
    vmin = sdd * fminf(fminf(v0, v1), fminf(v2, v3));
    vmax = sdd * fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
}

template <typename T>
__global__ __launch_bounds__(256) void k_cells(const ViewConst *__restrict__ views, DetConst dc,
                                               GridConst gc, int nu, int nv, int nviews,
                                               const T *__restrict__ r, T *__restrict__ cells,
                                               T step) {
    const int cx = (int)(blockIdx.x * CELL_BX + threadIdx.x) - 1;
    const int cy = (int)(blockIdx.y * CELL_BY + threadIdx.y) - 1;
    const int cz = (int)blockIdx.z - 1;
    const bool valid = cx < gc.nx && cy < gc.ny;
    const float cxf = (float)cx, cyf = (float)cy, czf = (float)cz;
    const double cxd = (double)cx, cyd = (double)cy, czd = (double)cz;
    // cell box in mm (voxel centres cx and cx+1, ...)
    const float xa = gc.x0 + (float)cx * gc.hx, xb = xa + gc.hx;
    const float ya = gc.y0 + (float)cy * gc.hy, yb = ya + gc.hy;
    const float za = gc.z0 + (float)cz * gc.hz, zb = za + gc.hz;
    const float margin = 0.01f;
    const float inv_au = 1.0f / dc.au, inv_av = 1.0f / dc.av;
    T acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = T(0);

    for (int k = 0; valid && k < nviews; ++k) {
        const ViewConst vc = views[k];
        float umin, umax, vmin, vmax;
        box_footprint(vc, dc.sdd, xa, xb, ya, yb, za, zb, umin, umax, vmin, vmax);
        int i0 = (int)ceilf(fmaxf((umin - dc.u0) * inv_au - margin, -1.0f));
        int i1 = (int)floorf(fminf((umax - dc.u0) * inv_au + margin, (float)nu));
        int j0 = (int)ceilf(fmaxf((vmin - dc.v0) * inv_av - margin, -1.0f));
        int j1 = (int)floorf(fminf((vmax - dc.v0) * inv_av + margin, (float)nv));
        i0 = i0 < 0 ? 0 : i0;
        j0 = j0 < 0 ? 0 : j0;
        i1 = i1 > nu - 1 ? nu - 1 : i1;
        j1 = j1 > nv - 1 ? nv - 1 : j1;
        const T *rk = r + (long long)k * nu * nv;
        for (int j = j0; j <= j1; ++j) {
            for (int i = i0; i <= i1; ++i) {
                // conservative candidate range from the float ray ...
                float Qf[3], Df[3];
                ray_setup(vc, dc, i, j, Qf, Df);
                float lo = -1e30f, hi = 1e30f, a = 0.0f, b = 0.0f;
                bool ok = axis_estimate(Qf[0], Df[0], cxf, lo, hi);
                ok = ok && axis_estimate(Qf[1], Df[1], cyf, a, b);
                lo = fmaxf(a, lo);
                hi = fminf(b, hi);
                ok = ok && axis_estimate(Qf[2], Df[2], czf, a, b);
                lo = fmaxf(a, lo);
                hi = fminf(b, hi);
                if (!ok || !(lo <= hi)) continue;
                const int n0 = clamp_to_int(-floor_t(-lo));  // ceil
                const int n1 = clamp_to_int(floor_t(hi));
                if (n0 > n1) continue;
                // ... then the exact cell test with the projector's coordinates
                double Q[3], D[3];
                ray_setup(vc, dc, i, j, Q, D);
                const T rv = rk[(long long)j * nu + i];
                double nf = (double)n0;
                for (int n = n0; n <= n1; ++n, nf += 1.0) {
                    const double q0 = sample_coord(nf, D[0], Q[0]);
                    const double q1 = sample_coord(nf, D[1], Q[1]);
                    const double q2 = sample_coord(nf, D[2], Q[2]);
                    const double f0 = floor_t(q0), f1 = floor_t(q1), f2 = floor_t(q2);
                    if (f0 != cxd || f1 != cyd || f2 != czd) continue;
                    const T wx = (T)(q0 - f0), wy = (T)(q1 - f1), wz = (T)(q2 - f2);
                    const T b1 = rv * wz, b0 = rv - b1;
                    const T a01 = b0 * wy, a00 = b0 - a01;
                    const T a11 = b1 * wy, a10 = b1 - a11;
                    T t;
                    t = a00 * wx; acc[0] += a00 - t; acc[1] += t;
                    t = a01 * wx; acc[2] += a01 - t; acc[3] += t;
                    t = a10 * wx; acc[4] += a10 - t; acc[5] += t;
                    t = a11 * wx; acc[6] += a11 - t; acc[7] += t;
                }
            }
        }
    }
    if (!valid) return;
    const long long ncell = (long long)(gc.nx + 1) * (gc.ny + 1) * (gc.nz + 1);
    const long long lin = (long long)(cx + 1) + (long long)(gc.nx + 1) * ((cy + 1) + (long long)(gc.ny + 1) * (cz + 1));
#pragma unroll
    for (int o = 0; o < 8; ++o) cells[o * ncell + lin] = acc[o] * step;
}

// Pass 2: out = sum of corner o of cell (v - o) over o in {0,1}^3,
// then out = f - tau * out when f is given.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(GridConst gc, const T *__restrict__ cells,
                                                const T *__restrict__ f, T tau,
                                                T *__restrict__ out) {
    const int ix = blockIdx.x * CELL_BX + threadIdx.x;
    const int iy = blockIdx.y * CELL_BY + threadIdx.y;
    const int iz = blockIdx.z;
    if (ix >= gc.nx || iy >= gc.ny) return;
    const long long cxn = gc.nx + 1, cxyn = cxn * (gc.ny + 1);
    const long long ncell = cxyn * (gc.nz + 1);
    // cell (ix - ox, iy - oy, iz - oz) is stored at (ix - ox + 1, ...)
    const long long base = (long long)(ix + 1) + cxn * (iy + 1) + cxyn * (iz + 1);
    T s = T(0);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        // voxel v is corner o of cell v - o (corners of cell c are c + o)
        s += cells[o * ncell + base - ox - oy * cxn - oz * cxyn];
    }
    const long long v = (long long)ix + (long long)gc.nx * (iy + (long long)gc.ny * iz);
    out[v] = f ? f[v] - tau * s : s;
}

}  // namespace

size_t cells_count(const cbct_plan &p) {
    return (size_t)8 * (p.g.nx + 1) * (p.g.ny + 1) * (p.g.nz + 1);
}

template <typename T>
hipError_t launch_backproject_cells(const cbct_plan &p, const T *r, T *cells, hipStream_t s) {
    dim3 grid((p.g.nx + 1 + CELL_BX - 1) / CELL_BX, (p.g.ny + 1 + CELL_BY - 1) / CELL_BY,
              p.g.nz + 1);
    hipLaunchKernelGGL(k_cells<T>, grid, dim3(CELL_BX, CELL_BY), 0, s, p.d_views, p.det, p.grid,
                       p.g.nu, p.g.nv, p.g.n_views, r, cells, (T)p.g.step);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_cells(const cbct_plan &p, const T *cells, const T *f, double tau,
                               T *out, hipStream_t s) {
    dim3 grid((p.g.nx + CELL_BX - 1) / CELL_BX, (p.g.ny + CELL_BY - 1) / CELL_BY, p.g.nz);
    hipLaunchKernelGGL(k_gather<T>, grid, dim3(CELL_BX, CELL_BY), 0, s, p.grid, cells, f, (T)tau,
                       out);
    return hipGetLastError();
}

template hipError_t launch_backproject_cells<float>(const cbct_plan &, const float *, float *,
                                                    hipStream_t);
template hipError_t launch_backproject_cells<double>(const cbct_plan &, const double *, double *,
                                                     hipStream_t);
template hipError_t launch_gather_cells<float>(const cbct_plan &, const float *, const float *,
                                               double, float *, hipStream_t);
template hipError_t launch_gather_cells<double>(const cbct_plan &, const double *,
                                                const double *, double, double *, hipStream_t);

}  // namespace cbct
