// Transpose of the projector, P^T, in gather form without atomics.
//
// The paper computes the gradient of E2 per voxel by a gather (Eq. (2)) to
// avoid the write conflicts of the scattering matrix transpose.  Here the
// gather is the EXACT transpose of the discrete projector, organised by
// interpolation cell rather than by voxel:
//
//   * a cell c = (cx, cy, cz), c_a in [-1, N_a - 1], is the box between
//     voxel centres c and c + 1; every projector sample lies in exactly one
//     cell, the one given by the projector's own cell arithmetic;
//   * pass 1 (one lane per cell, a workgroup per 8x8x4 brick of cells): for
//     every view the workgroup projects its brick on the detector and
//     stages the ray direction (double) and residual of every pixel in that
//     footprint in LDS; each lane then visits the pixels whose rays can
//     cross its cell, enumerates the samples of each such ray that fall in
//     the cell, and accumulates r * (trilinear corner weight) into eight
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

constexpr int CB_X = 8, CB_Y = 8, CB_Z = 4;  // cells per workgroup
constexpr int TABLE = 768;                    // pixels staged per view
constexpr int G_BX = 64, G_BY = 4;            // pass-2 block

// Staged per pixel: the ray increment D in double (exact cell test), the
// reciprocal of its float rounding (range estimate; 1e30 stands for the
// reciprocal of an exactly zero component) and the residual.
struct PixelRay {
    double D[3];
    float inv[3];
    float r;
};

__device__ __forceinline__ float inv_or_huge(float d) {
    return d != 0.0f ? __builtin_amdgcn_rcpf(d) : 1e30f;
}

// Per-lane, per-view constants of the candidate range of cell c: along
// axis a the samples with coordinate in [c_a, c_a + 1) lie between
// (c_a - Q_a)/D_a and (c_a + 1 - Q_a)/D_a.  The float Q and D differ from
// the double ones by at most ~1e-6 relative, which moves those bounds by at
// most 1e-6 (|Q| + |c| + 1)/|D|; the range is widened by four times that
// plus 1e-3 (covers the rounding of the float estimate itself).
struct CellRange {
    float cq[3];  // c_a - Q_a
    float K[3];   // 4e-6 (|Q_a| + |c_a| + 1)
};

__device__ __forceinline__ CellRange cell_range(const float Qf[3], float cx, float cy, float cz) {
    CellRange cr;
    const float c[3] = {cx, cy, cz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cr.cq[a] = c[a] - Qf[a];
        cr.K[a] = 4e-6f * (fabsf(Qf[a]) + fabsf(c[a]) + 1.0f);
    }
    return cr;
}

// Candidate samples [n0, n1] of the ray with reciprocal increments inv.
__device__ __forceinline__ bool candidates_inv(const CellRange &cr, const float inv[3], int &n0,
                                               int &n1) {
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float t0 = cr.cq[a] * inv[a];
        const float t1 = t0 + inv[a];
        const float m = __builtin_fmaf(cr.K[a], fabsf(inv[a]), 1e-3f);
        lo[a] = fminf(t0, t1) - m;
        hi[a] = fmaxf(t0, t1) + m;
    }
    const float l = fmaxf(fmaxf(lo[0], lo[1]), lo[2]);
    const float h = fminf(fminf(hi[0], hi[1]), hi[2]);
    if (!(l <= h)) return false;
    n0 = clamp_to_int(-floor_t(-l));
    n1 = clamp_to_int(floor_t(h));
    return n0 <= n1;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

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
    const float u00 = n00 * rcp(d00), u10 = n10 * rcp(d10);
    const float u01 = n01 * rcp(d01), u11 = n11 * rcp(d11);
    umin = sdd * fminf(fminf(u00, u10), fminf(u01, u11));
    umax = sdd * fmaxf(fmaxf(u00, u10), fmaxf(u01, u11));
    const float ia = rcp(fminf(fminf(d00, d10), fminf(d01, d11)));
    const float ib = rcp(fmaxf(fmaxf(d00, d10), fmaxf(d01, d11)));
    const float v0 = za * ia, v1 = za * ib, v2 = zb * ia, v3 = zb * ib;
    vmin = sdd * fminf(fminf(v0, v1), fminf(v2, v3));
    vmax = sdd * fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
}

// Pixel index range [i0, i1] x [j0, j1] whose centres fall inside the
// detector rectangle [umin, umax] x [vmin, vmax] widened by 0.01 pixel.
__device__ __forceinline__ void pixel_range(const DetConst &dc, int nu, int nv, float umin,
                                            float umax, float vmin, float vmax, int &i0, int &i1,
                                            int &j0, int &j1) {
    const float margin = 0.01f;
    const float iau = rcp(dc.au), iav = rcp(dc.av);
    i0 = (int)ceilf(fmaxf((umin - dc.u0) * iau - margin, -1.0f));
    i1 = (int)floorf(fminf((umax - dc.u0) * iau + margin, (float)nu));
    j0 = (int)ceilf(fmaxf((vmin - dc.v0) * iav - margin, -1.0f));
    j1 = (int)floorf(fminf((vmax - dc.v0) * iav + margin, (float)nv));
    i0 = i0 < 0 ? 0 : i0;
    j0 = j0 < 0 ? 0 : j0;
    i1 = i1 > nu - 1 ? nu - 1 : i1;
    j1 = j1 > nv - 1 ? nv - 1 : j1;
}

// Accumulate r * corner weights of sample weights (wx, wy, wz).
template <typename T>
__device__ __forceinline__ void add_corners(T acc[8], T rv, T wx, T wy, T wz) {
    const T b1 = rv * wz, b0 = rv - b1;
    const T a01 = b0 * wy, a00 = b0 - a01;
    const T a11 = b1 * wy, a10 = b1 - a11;
    T t;
    t = a00 * wx; acc[0] += a00 - t; acc[1] += t;
    t = a01 * wx; acc[2] += a01 - t; acc[3] += t;
    t = a10 * wx; acc[4] += a10 - t; acc[5] += t;
    t = a11 * wx; acc[6] += a11 - t; acc[7] += t;
}

// Samples n0..n1 of the ray (Qd, D) that fall in cell (cx, cy, cz): the
// projector's cell arithmetic decides membership.
template <typename T>
__device__ __forceinline__ void cell_samples(T acc[8], T rv, const double Qd[3],
                                             const double D[3], int n0, int n1, int cx, int cy,
                                             int cz) {
    if constexpr (sizeof(T) == 4) {
#pragma clang fp contract(off)
        float Df[3];
        to_float3(D, Df);
        int ns = n0 & ~(SEG - 1);
        SegOrigin o = seg_origin(Qd, D, ns);
        // The projector puts sample m of the segment in cell I + floor(l) with
        // l = fma(m, Df, f).  For the integer L = c - I, floor(l) == L exactly
        // when L <= l < L + 1, and the weight l - floor(l) is then l - L.
        float L[3], H[3];
        auto bounds = [&]() {
            L[0] = (float)(cx - o.I[0]);
            L[1] = (float)(cy - o.I[1]);
            L[2] = (float)(cz - o.I[2]);
            H[0] = L[0] + 1.0f;
            H[1] = L[1] + 1.0f;
            H[2] = L[2] + 1.0f;
        };
        bounds();
        float m = (float)(n0 - ns);
        for (int n = n0; n <= n1; ++n, m += 1.0f) {
            if (n == ns + SEG) {
                ns += SEG;
                m = 0.0f;
                o = seg_origin(Qd, D, ns);
                bounds();
            }
            const float lx = __builtin_fmaf(m, Df[0], o.f[0]);
            const float ly = __builtin_fmaf(m, Df[1], o.f[1]);
            const float lz = __builtin_fmaf(m, Df[2], o.f[2]);
            const bool in = (lx >= L[0]) & (lx < H[0]) & (ly >= L[1]) & (ly < H[1]) &
                            (lz >= L[2]) & (lz < H[2]);
            if (!in) continue;
            add_corners<T>(acc, rv, lx - L[0], ly - L[1], lz - L[2]);
        }
    } else {
        double nf = (double)n0;
        for (int n = n0; n <= n1; ++n, nf += 1.0) {
            const double q0 = sample_coord(nf, D[0], Qd[0]);
            const double q1 = sample_coord(nf, D[1], Qd[1]);
            const double q2 = sample_coord(nf, D[2], Qd[2]);
            const double f0 = floor_t(q0), f1 = floor_t(q1), f2 = floor_t(q2);
            if ((int)f0 != cx || (int)f1 != cy || (int)f2 != cz) continue;
            add_corners<T>(acc, rv, (T)(q0 - f0), (T)(q1 - f1), (T)(q2 - f2));
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cells(const ViewConst *__restrict__ views, DetConst dc,
                                               GridConst gc, int nu, int nv, int nviews,
                                               const T *__restrict__ r, T *__restrict__ cells,
                                               T step) {
    __shared__ PixelRay table[TABLE];
    const int tid = threadIdx.x;
    const int bx0 = blockIdx.x * CB_X - 1, by0 = blockIdx.y * CB_Y - 1,
              bz0 = blockIdx.z * CB_Z - 1;  // first cell of the brick
    const int cx = bx0 + (tid & (CB_X - 1));
    const int cy = by0 + ((tid / CB_X) & (CB_Y - 1));
    const int cz = bz0 + tid / (CB_X * CB_Y);
    const bool valid = cx < gc.nx && cy < gc.ny && cz < gc.nz;
    // brick box (cells up to the last one of the grid)
    const int bx1 = min(bx0 + CB_X - 1, gc.nx - 1), by1 = min(by0 + CB_Y - 1, gc.ny - 1),
              bz1 = min(bz0 + CB_Z - 1, gc.nz - 1);
    const float Bxa = gc.x0 + (float)bx0 * gc.hx, Bxb = gc.x0 + (float)(bx1 + 1) * gc.hx;
    const float Bya = gc.y0 + (float)by0 * gc.hy, Byb = gc.y0 + (float)(by1 + 1) * gc.hy;
    const float Bza = gc.z0 + (float)bz0 * gc.hz, Bzb = gc.z0 + (float)(bz1 + 1) * gc.hz;
    // this lane's cell box (same expressions as the brick box, so shared
    // faces round identically)
    const float xa = gc.x0 + (float)cx * gc.hx, xb = gc.x0 + (float)(cx + 1) * gc.hx;
    const float ya = gc.y0 + (float)cy * gc.hy, yb = gc.y0 + (float)(cy + 1) * gc.hy;
    const float za = gc.z0 + (float)cz * gc.hz, zb = gc.z0 + (float)(cz + 1) * gc.hz;
    const float cxf = (float)cx, cyf = (float)cy, czf = (float)cz;
    T acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = T(0);

    for (int k = 0; k < nviews; ++k) {
        const ViewConst vc = views[k];
        const T *rk = r + (long long)k * nu * nv;
        // workgroup footprint, identical in every lane
        float umin, umax, vmin, vmax;
        box_footprint(vc, dc.sdd, Bxa, Bxb, Bya, Byb, Bza, Bzb, umin, umax, vmin, vmax);
        int bi0, bi1, bj0, bj1;
        pixel_range(dc, nu, nv, umin, umax, vmin, vmax, bi0, bi1, bj0, bj1);
        const int bw = bi1 - bi0 + 1, bh = bj1 - bj0 + 1;
        if (bw <= 0 || bh <= 0) continue;  // uniform: the brick misses the detector
        const bool staged = bw * bh <= TABLE;
        if (staged) {
            __syncthreads();  // readers of the previous view are done
            for (int t = tid; t < bw * bh; t += 256) {
                const int j = bj0 + t / bw, i = bi0 + t % bw;
                double Q[3], D[3];
                ray_setup(vc, dc, i, j, Q, D);
                float Df[3];
                to_float3(D, Df);
                table[t].D[0] = D[0];
                table[t].D[1] = D[1];
                table[t].D[2] = D[2];
                table[t].inv[0] = inv_or_huge(Df[0]);
                table[t].inv[1] = inv_or_huge(Df[1]);
                table[t].inv[2] = inv_or_huge(Df[2]);
                table[t].r = (float)rk[(long long)j * nu + i];
            }
            __syncthreads();
        }
        if (!valid) continue;
        box_footprint(vc, dc.sdd, xa, xb, ya, yb, za, zb, umin, umax, vmin, vmax);
        int i0, i1, j0, j1;
        pixel_range(dc, nu, nv, umin, umax, vmin, vmax, i0, i1, j0, j1);
        // the cell lies in the brick: keep its pixels inside the staged
        // rectangle (they differ at most by rounding, inside the margin)
        i0 = max(i0, bi0);
        i1 = min(i1, bi1);
        j0 = max(j0, bj0);
        j1 = min(j1, bj1);
        const float Qf[3] = {vc.Q[0], vc.Q[1], vc.Q[2]};
        const CellRange cr = cell_range(Qf, cxf, cyf, czf);
        if (staged) {
            // (the cell's rectangle is nearly its exact footprint: almost
            // every pixel visited has samples in the cell).  One flat loop
            // over the rectangle: lanes with rectangles of different shapes
            // then diverge only in the total pixel count.
            const int w = i1 - i0 + 1, h = j1 - j0 + 1;
            const int npix = (w > 0 && h > 0) ? w * h : 0;
            int i = i0, j = j0;
            const PixelRay *row = table + (j0 - bj0) * bw - bi0;
            for (int q = 0; q < npix; ++q) {
                const PixelRay &pr = row[i];
                const int pi = i, pj = j;
                if (++i > i1) {
                    i = i0;
                    ++j;
                    row += bw;
                }
                const float inv[3] = {pr.inv[0], pr.inv[1], pr.inv[2]};
                int n0, n1;
                if (!candidates_inv(cr, inv, n0, n1)) continue;
                const double D[3] = {pr.D[0], pr.D[1], pr.D[2]};
                // double data: residual at full precision from memory
                const T rv = sizeof(T) == 8 ? rk[(long long)pj * nu + pi] : (T)pr.r;
                cell_samples<T>(acc, rv, vc.Qd, D, n0, n1, cx, cy, cz);
            }
            continue;
        }
        for (int j = j0; j <= j1; ++j) {
            for (int i = i0; i <= i1; ++i) {
                int n0, n1;
                {
                    double Qd[3], D[3];
                    ray_setup(vc, dc, i, j, Qd, D);
                    float Df[3];
                    to_float3(D, Df);
                    const float inv[3] = {inv_or_huge(Df[0]), inv_or_huge(Df[1]),
                                          inv_or_huge(Df[2])};
                    if (!candidates_inv(cr, inv, n0, n1)) continue;
                    cell_samples<T>(acc, rk[(long long)j * nu + i], vc.Qd, D, n0, n1, cx, cy,
                                    cz);
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
    const int ix = blockIdx.x * G_BX + threadIdx.x;
    const int iy = blockIdx.y * G_BY + threadIdx.y;
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
    dim3 grid((p.g.nx + 1 + CB_X - 1) / CB_X, (p.g.ny + 1 + CB_Y - 1) / CB_Y,
              (p.g.nz + 1 + CB_Z - 1) / CB_Z);
    hipLaunchKernelGGL(k_cells<T>, grid, dim3(256), 0, s, p.d_views, p.det, p.grid, p.g.nu,
                       p.g.nv, p.g.n_views, r, cells, (T)p.g.step);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_cells(const cbct_plan &p, const T *cells, const T *f, double tau,
                               T *out, hipStream_t s) {
    dim3 grid((p.g.nx + G_BX - 1) / G_BX, (p.g.ny + G_BY - 1) / G_BY, p.g.nz);
    hipLaunchKernelGGL(k_gather<T>, grid, dim3(G_BX, G_BY), 0, s, p.grid, cells, f, (T)tau, out);
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
