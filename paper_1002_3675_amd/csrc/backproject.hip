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
//   * preparation (geometry only, once per plan or workspace): the ray
//     increment of every pixel of every view, and every brick's pixel
//     rectangle per view (its footprint on the detector);
//   * pass 1 (one lane per cell, a workgroup per 16x16x1 brick of cells):
//     for every view the workgroup stages, per pixel of its brick's
//     footprint, the candidate-range terms, the segment origin of the ray
//     in the brick and the residual in LDS; each lane then visits the
//     pixels whose rays can cross its cell, enumerates the samples of each
//     such ray that fall in the cell, and accumulates r * (trilinear
//     corner weight), in xy-moment form, into eight register accumulators;
//   * pass 2 (one lane per voxel): sum the matching corner of the eight
//     cells that share the voxel, optionally fused with Step 1 of
//     Algorithm A1, g = f - tau * P^T r.
//
// Each (ray, sample) is visited once instead of eight times (once per
// trilinear tap), every sum has a fixed order, and no lane writes memory
// another lane writes.
#include "ray.hpp"

#ifndef CBCT_CELL_TABLE
#define CBCT_CELL_TABLE 344
#endif

namespace cbct {

namespace {

constexpr int CB_X = 16, CB_Y = 16, CB_Z = 1;  // cells per workgroup: one z layer
constexpr int TABLE = CBCT_CELL_TABLE;         // pixels staged per view (60 B each)
constexpr int G_BX = 64, G_BY = 4;            // pass-2 block

// Row pitch (in elements) of the cell corner-sum array: nx + 1 cells
// rounded up to 32, so that every brick row of cells (16 consecutive x
// cells, starting at a multiple of 16) is a whole, aligned 64-byte segment
// for float and the rows of a plane start on 128-byte boundaries.
__host__ __device__ __forceinline__ long long cell_pitch(int nx) {
    return ((long long)nx + 1 + 31) & ~31LL;
}

// Ray table entry per pixel and view (prepared once): the ray increment D
// in double (segment origins).  Readers form the reciprocals of its float
// rounding for the range estimates themselves (ray_inv).  24 bytes.
struct PixelRay {
    double D[3];
};

// LDS entry per footprint pixel of the current view, in two parts.
//
// StagedRange serves the candidate test every cell of the brick makes for
// this pixel.  Along axis a the samples with coordinate in [c_a, c_a + 1)
// lie between (c_a - Q_a)/D_a and (c_a + 1 - Q_a)/D_a.  The float Q and D
// differ from the double ones by at most ~1e-6 relative, which moves these
// bounds by at most 1e-6 (|Q_a| + |c_a| + 1) |inv_a| (inv = 1/D_f); a
// margin m_a = K_a |inv_a| + 1e-3 with K_a = 4e-6 (|Q_a| + max |c_a| over
// the brick + 1) covers four times that plus the rounding of the float
// estimate itself.  With the cell's cq_a = c_a - Q_a (float) the widened
// bounds are
//     lo_a = fma(cq_a, inv_a, min(0, inv_a) - m_a),
//     hi_a = lo_a + |inv_a| (1 + 2 K_a) + 2e-3,
// and lo[a] holds the additive term of lo_a (a = x, y).  Every cell of the
// brick lies in the same z layer, so the z bounds are the same for all of
// them: zlo, zhi.  24 bytes.
//
// StagedWalk serves the cells with candidates: the origin (I, f) of the
// segment sq * SEG that holds the ray's first sample in the brick, as the
// projector computes it; D_f = (float)D; the residual.  Cells whose
// candidates start in another segment compute that segment's origin from
// the ray table.  Grid dimensions below 32000 keep I (within SEG/2 + 2
// cells of the brick) in a short.  36 bytes.
struct StagedRange {
    float inv[2];
    float lo[2];
    float zlo, zhi;
};

struct StagedWalk {
    float f[3];
    float Df[3];
    float r;
    short I[3];
    short sq;
};

// Both parts of a pixel's entry, side by side: one pointer reaches both.
struct StagedEntry {
    StagedRange rg;
    StagedWalk wk;
};
static_assert(sizeof(StagedEntry) == 60, "60-byte LDS entries");

__device__ __forceinline__ float inv_or_huge(float d) {
    return d != 0.0f ? __builtin_amdgcn_rcpf(d) : 1e30f;
}

// Reciprocals of the float rounding of a ray's increment (1e30 stands for
// the reciprocal of an exactly zero component).
__device__ __forceinline__ void ray_inv(const PixelRay &g, float inv[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) inv[a] = inv_or_huge((float)g.D[a]);
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

// Float accumulation of r * corner weights in xy-moment form: for each z
// corner oz the cell keeps S = sum b, X = sum b wx, Y = sum b wy and
// XY = sum b wx wy, b = r * (z weight); the corners are (S - X) - (Y - XY),
// X - XY, Y - XY and XY (moments_to_corners).  12 operations per sample
// instead of 22.  The differences carry an absolute error of a few ulp of
// S, the cell's mass on that z face, which is at most the sum over the
// corners the voxel gather adds it to.
__device__ __forceinline__ void add_moments(float acc[8], float rv, float wx, float wy,
                                            float wz) {
    const float b1 = rv * wz, b0 = rv - b1;
    acc[0] += b0;
    acc[1] = __builtin_fmaf(b0, wx, acc[1]);
    acc[2] = __builtin_fmaf(b0, wy, acc[2]);
    acc[3] = __builtin_fmaf(b0 * wx, wy, acc[3]);
    acc[4] += b1;
    acc[5] = __builtin_fmaf(b1, wx, acc[5]);
    acc[6] = __builtin_fmaf(b1, wy, acc[6]);
    acc[7] = __builtin_fmaf(b1 * wx, wy, acc[7]);
}

// Corner sums (index ox + 2 oy + 4 oz) from the xy-moments of add_moments.
__device__ __forceinline__ void moments_to_corners(const float m[8], float c[8]) {
#pragma unroll
    for (int z = 0; z < 2; ++z) {
        const float S = m[4 * z], X = m[4 * z + 1], Y = m[4 * z + 2], XY = m[4 * z + 3];
        c[4 * z + 0] = (S - X) - (Y - XY);
        c[4 * z + 1] = X - XY;
        c[4 * z + 2] = Y - XY;
        c[4 * z + 3] = XY;
    }
}

// Where a pixel's ray-table entry is, computed only on the rare path that
// needs the ray's double increment.  The pixel index passes through an
// empty asm statement first, so the compiler cannot hoist the 64-bit
// address arithmetic out of that path into every visit.
struct RayRef {
    const PixelRay *view;  // the view's table
    int nu, i, j;
    __device__ __forceinline__ const PixelRay *get() const {
        int jj = j, ii = i;
        asm volatile("" : "+v"(jj), "+v"(ii));
        return view + ((long long)jj * nu + ii);
    }
};

// Candidate samples of a ray in cell (cx, cy, cz), float data: sample
// indices sf * SEG + m for m from m0 to mlast (integer-valued floats, sf the
// segment number, m0 < SEG; mlast may run into later segments); o is the
// origin of segment sf.  A later segment's origin is computed from the
// ray's double increment in the ray table.  The projector's own cell
// arithmetic decides membership; a candidate outside the cell adds zero (no
// branch in the loop body).
__device__ __forceinline__ void cell_samples_f(float acc[8], float rv, const double Qd[3],
                                               const RayRef &ray, SegOrigin o, float sf,
                                               const float Df[3], float m, float mlast, int cx,
                                               int cy, int cz) {
#pragma clang fp contract(off)
    // The projector puts sample m of the segment in cell I + floor(l) with
    // l = fma(m, Df, f), weight l - floor(l): the sample is in cell c when
    // floor(l) == L = c - I on every axis, and its weight is then l - L.
    // With L an integer, w = l - L rounds to itself except for l in
    // [-2^-25, 0) with L = -1, where it rounds up to 1; rounding keeps w's
    // sign and its order against 1.  So floor(l) == L exactly when w, read as
    // an unsigned integer, is below that of 1.0f (a negative w has its sign
    // bit set, l - L = 0 gives +0), except when some w is exactly 1: then
    // floor decides, as in the projector, in a second pass over the
    // segment's candidates.
    float L[3];
    auto bounds = [&]() {
        L[0] = (float)(cx - o.I[0]);
        L[1] = (float)(cy - o.I[1]);
        L[2] = (float)(cz - o.I[2]);
    };
    bounds();
    constexpr unsigned ONE = 0x3f800000u;  // 1.0f
    for (;;) {
        // samples up to the end of this segment (float counts are exact)
        const float mend = __builtin_amdgcn_fmed3f(mlast, 0.0f, (float)(SEG - 1));  // mlast >= 0
        const float mstart = m;
        bool edge = false;  // some sample had a weight of exactly 1
        for (; m <= mend; m += 1.0f) {
            const float wx = __builtin_fmaf(m, Df[0], o.f[0]) - L[0];
            const float wy = __builtin_fmaf(m, Df[1], o.f[1]) - L[1];
            const float wz = __builtin_fmaf(m, Df[2], o.f[2]) - L[2];
            const unsigned wmax = max(max(__builtin_bit_cast(unsigned, wx),
                                          __builtin_bit_cast(unsigned, wy)),
                                      __builtin_bit_cast(unsigned, wz));
            add_moments(acc, wmax < ONE ? rv : 0.0f, wx, wy, wz);
            edge |= wmax == ONE;
        }
        if (edge) {
            // rare: add the samples with a weight of 1 that floor puts in
            // the cell (after the others: the order of the sum changes, not
            // its terms)
            for (float mm = mstart; mm <= mend; mm += 1.0f) {
                const float lx = __builtin_fmaf(mm, Df[0], o.f[0]);
                const float ly = __builtin_fmaf(mm, Df[1], o.f[1]);
                const float lz = __builtin_fmaf(mm, Df[2], o.f[2]);
                const float wx = lx - L[0], wy = ly - L[1], wz = lz - L[2];
                const unsigned wmax = max(max(__builtin_bit_cast(unsigned, wx),
                                              __builtin_bit_cast(unsigned, wy)),
                                          __builtin_bit_cast(unsigned, wz));
                const bool in = (__builtin_floorf(lx) == L[0]) &
                                (__builtin_floorf(ly) == L[1]) & (__builtin_floorf(lz) == L[2]);
                if (wmax == ONE && in) add_moments(acc, rv, wx, wy, wz);
            }
        }
        if (mlast <= (float)(SEG - 1)) return;
        // rare: the cell's samples of this ray run into the next segment
        sf += 1.0f;
        m = 0.0f;
        mlast -= (float)SEG;
        const PixelRay *gray = ray.get();
        const double D[3] = {gray->D[0], gray->D[1], gray->D[2]};
        o = seg_origin(Qd, D, (int)sf * SEG);
        bounds();
    }
}

// The same for double data: every sample in double, no segments.
__device__ __forceinline__ void cell_samples_d(double acc[8], double rv, const double Qd[3],
                                               const double D[3], int n0, int n1, int cx,
                                               int cy, int cz) {
    double nf = (double)n0;
    for (int n = n0; n <= n1; ++n, nf += 1.0) {
        const double q0 = sample_coord(nf, D[0], Qd[0]);
        const double q1 = sample_coord(nf, D[1], Qd[1]);
        const double q2 = sample_coord(nf, D[2], Qd[2]);
        const double f0 = floor_t(q0), f1 = floor_t(q1), f2 = floor_t(q2);
        if ((int)f0 != cx || (int)f1 != cy || (int)f2 != cz) continue;
        add_corners<double>(acc, rv, q0 - f0, q1 - f1, q2 - f2);
    }
}

// Geometry-only preparation, once per plan and workspace:
//   k_rays:        the increment D (double) and its float reciprocals of the
//                  ray through every pixel of every view;
//   k_brick_rects: for every view and brick, the pixel rectangle whose rays
//                  can reach the brick (its staged footprint).
__global__ __launch_bounds__(256) void k_rays(const ViewConst *__restrict__ views, DetConst dc,
                                              int nu, int nv, PixelRay *__restrict__ rays) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= nu || j >= nv) return;
    double Q[3], D[3];
    ray_setup(views[k], dc, i, j, Q, D);
    PixelRay e;
    e.D[0] = D[0];
    e.D[1] = D[1];
    e.D[2] = D[2];
    rays[((long long)k * nv + j) * nu + i] = e;
}

// First cell and the box (mm) of brick (bxi, byi, bzi); the last brick of an
// axis ends at the grid's last cell.  Cells c_a run from -1 to N_a - 1.
struct BrickBox {
    int c0[3];
    float lo[3], hi[3];
};

__device__ __forceinline__ BrickBox brick_box(const GridConst &gc, int bxi, int byi, int bzi) {
    BrickBox b;
    b.c0[0] = bxi * CB_X - 1;
    b.c0[1] = byi * CB_Y - 1;
    b.c0[2] = bzi * CB_Z - 1;
    const int x1 = min(b.c0[0] + CB_X - 1, gc.nx - 1), y1 = min(b.c0[1] + CB_Y - 1, gc.ny - 1),
              z1 = min(b.c0[2] + CB_Z - 1, gc.nz - 1);
    b.lo[0] = gc.x0 + (float)b.c0[0] * gc.hx;
    b.hi[0] = gc.x0 + (float)(x1 + 1) * gc.hx;
    b.lo[1] = gc.y0 + (float)b.c0[1] * gc.hy;
    b.hi[1] = gc.y0 + (float)(y1 + 1) * gc.hy;
    b.lo[2] = gc.z0 + (float)b.c0[2] * gc.hz;
    b.hi[2] = gc.z0 + (float)(z1 + 1) * gc.hz;
    return b;
}

__global__ __launch_bounds__(256) void k_brick_rects(const ViewConst *__restrict__ views,
                                                     DetConst dc, GridConst gc, int nu, int nv,
                                                     int nbx, int nby, int nbz, int nviews,
                                                     int4 *__restrict__ rects) {
    const long long nb = (long long)nbx * nby * nbz;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nb * nviews) return;
    const int k = (int)(t / nb);
    const int b = (int)(t - (long long)k * nb);
    const int bxi = b % nbx, byi = (b / nbx) % nby, bzi = b / (nbx * nby);
    const BrickBox bb = brick_box(gc, bxi, byi, bzi);
    float umin, umax, vmin, vmax;
    box_footprint(views[k], dc.sdd, bb.lo[0], bb.hi[0], bb.lo[1], bb.hi[1], bb.lo[2], bb.hi[2],
                  umin, umax, vmin, vmax);
    int i0, i1, j0, j1;
    pixel_range(dc, nu, nv, umin, umax, vmin, vmax, i0, i1, j0, j1);
    rects[t] = make_int4(i0, i1, j0, j1);
}

// Accumulate the samples of one ray (residual rv) that fall in the cell:
// from the LDS entries (float data) or from the ray table (either type).
__device__ __forceinline__ void visit_staged(float acc[8], const float cq[2], const float kw[2],
                                             const StagedEntry &en, const RayRef &ray,
                                             const double Qd[3], int cx, int cy, int cz) {
    const StagedRange &er = en.rg;
    const float lx = __builtin_fmaf(cq[0], er.inv[0], er.lo[0]);
    const float ly = __builtin_fmaf(cq[1], er.inv[1], er.lo[1]);
    const float hx = lx + __builtin_fmaf(fabsf(er.inv[0]), kw[0], 2e-3f);
    const float hy = ly + __builtin_fmaf(fabsf(er.inv[1]), kw[1], 2e-3f);
    const float lo = fmaxf(fmaxf(lx, ly), er.zlo);
    const float hi = fminf(fminf(hx, hy), er.zhi);
    if (!(lo <= hi)) return;
    // first and last candidate sample, clamped as clamp_to_int clamps, kept
    // in float (integers below 2^24 are exact)
    const float n0 = __builtin_amdgcn_fmed3f(-floor_t(-lo), -4.0f, (float)(1 << 24));
    const float n1 = __builtin_amdgcn_fmed3f(floor_t(hi), -4.0f, (float)(1 << 24));
    if (!(n0 <= n1)) return;
    const float sf = floor_t(n0 * (1.0f / SEG));  // segment number
    const StagedWalk &e = en.wk;
    SegOrigin o;
    if ((int)sf == (int)e.sq) {
        o.I[0] = e.I[0];
        o.I[1] = e.I[1];
        o.I[2] = e.I[2];
        o.f[0] = e.f[0];
        o.f[1] = e.f[1];
        o.f[2] = e.f[2];
    } else {
        const PixelRay *gray = ray.get();
        const double D[3] = {gray->D[0], gray->D[1], gray->D[2]};
        o = seg_origin(Qd, D, (int)sf * SEG);
    }
    const float Df[3] = {e.Df[0], e.Df[1], e.Df[2]};
    cell_samples_f(acc, e.r, Qd, ray, o, sf, Df, __builtin_fmaf(sf, -(float)SEG, n0),
                   __builtin_fmaf(sf, -(float)SEG, n1), cx, cy, cz);
}

template <typename T>
__device__ __forceinline__ void visit_global(T acc[8], const CellRange &cr, const RayRef &ray,
                                             T rv, const double Qd[3], int cx, int cy, int cz) {
    const PixelRay *gray = ray.get();
    const PixelRay g = *gray;
    float inv[3];
    ray_inv(g, inv);
    int n0, n1;
    if (!candidates_inv(cr, inv, n0, n1)) return;
    const double D[3] = {g.D[0], g.D[1], g.D[2]};
    if constexpr (sizeof(T) == 4) {
        const int ns = n0 & ~(SEG - 1);
        float Df[3];
        to_float3(D, Df);
        cell_samples_f(acc, rv, Qd, ray, seg_origin(Qd, D, ns), (float)(ns / SEG), Df,
                       (float)(n0 - ns), (float)(n1 - ns), cx, cy, cz);
    } else {
        cell_samples_d(acc, rv, Qd, D, n0, n1, cx, cy, cz);
    }
}

// Workgroups of 256 lanes, one per brick.  Seven share a CU: 22.9 KB of
// LDS (60 bytes per staged pixel and the brick's projected corners) and at
// most 72 VGPRs.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_cells(const ViewConst *__restrict__ views, DetConst dc,
                                               GridConst gc, int nu, int nv, int nviews,
                                               const PixelRay *__restrict__ rays,
                                               const int4 *__restrict__ rects,
                                               const T *__restrict__ r, T *__restrict__ cells,
                                               T step) {
    __shared__ StagedEntry table[TABLE];
    __shared__ float2 corner[(CB_X + 1) * (CB_Y + 1)];
    const int tid = threadIdx.x;
    // bricks x-fastest, then y, then z; each XCD takes one contiguous range,
    // so the bricks resident on an XCD at a time are neighbours whose
    // footprints (ray table rows) overlap in its L2
    const int nbx = (gc.nx + 1 + CB_X - 1) / CB_X, nby = (gc.ny + 1 + CB_Y - 1) / CB_Y;
    const int nb = gridDim.x;
    const int brick = xcd_tile(blockIdx.x, nb);
    const BrickBox bb = brick_box(gc, brick % nbx, (brick / nbx) % nby, brick / (nbx * nby));
    const int cx = bb.c0[0] + (tid % CB_X);
    const int cy = bb.c0[1] + (tid / CB_X) % CB_Y;
    const int cz = bb.c0[2] + tid / (CB_X * CB_Y);
    const bool valid = cx < gc.nx && cy < gc.ny && cz < gc.nz;
    // the brick's single z layer (CB_Z = 1): cell cz0 = blo[2] below
    static_assert(CB_Z == 1, "the staged z bounds assume one z layer per brick");
    T acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = T(0);

    for (int k = 0; k < nviews; ++k) {
        // Per-view copies of brick and lane constants.  They are formed
        // again in every view from copies passed through an empty asm
        // statement: held across the view loop instead, they would be
        // spilled under the register budget.
        int c0[3] = {bb.c0[0], bb.c0[1], bb.c0[2]}, lx = cx, ly = cy;
        asm volatile("" : "+s"(c0[0]), "+s"(c0[1]), "+s"(c0[2]), "+v"(lx), "+v"(ly));
        // the brick in index coordinates: cells c0 .. c1 cover [c0, c1 + 1)
        const float blo[3] = {(float)c0[0], (float)c0[1], (float)c0[2]};
        const float bhi[3] = {(float)min(c0[0] + CB_X, gc.nx), (float)min(c0[1] + CB_Y, gc.ny),
                              (float)min(c0[2] + CB_Z, gc.nz)};
        // this lane's cell faces in z (same expressions as the brick box)
        const float za = gc.z0 + (float)cz * gc.hz, zb = gc.z0 + (float)(cz + 1) * gc.hz;
        const float cxf = (float)lx, cyf = (float)ly, czf = (float)cz;
        // largest |c_a| over the brick's cells, for the staged range margins
        const float cmax[3] = {fmaxf(fabsf(blo[0]), fabsf(bhi[0])),
                               fmaxf(fabsf(blo[1]), fabsf(bhi[1])),
                               fmaxf(fabsf(blo[2]), fabsf(bhi[2]))};
        const ViewConst vc = views[k];
        const long long vbase = (long long)k * nu * nv;
        const T *rk = r + vbase;
        const PixelRay *raysk = rays + vbase;
        // the brick's footprint, identical in every lane
        const int4 rect = rects[(long long)k * nb + brick];
        const int bi0 = rect.x, bi1 = rect.y, bj0 = rect.z, bj1 = rect.w;
        const int bw = bi1 - bi0 + 1, bh = bj1 - bj0 + 1;
        if (bw <= 0 || bh <= 0) continue;  // uniform: the brick misses the detector
        // float data stages the footprint in LDS; double reads the ray
        // table and the residual at full precision from memory
        const bool staged = sizeof(T) == 4 && bw * bh <= TABLE;
        __syncthreads();  // readers of the previous view are done
        // the brick's (CB_X + 1) x (CB_Y + 1) cell corners in the xy plane,
        // projected: u / sdd and 1 / depth (the corner expressions of
        // box_footprint, shared by the cells of every layer)
        for (int t = tid; t < (CB_X + 1) * (CB_Y + 1); t += 256) {
            const int a = t % (CB_X + 1), b = t / (CB_X + 1);
            const float x = gc.x0 + (float)(bb.c0[0] + a) * gc.hx;
            const float y = gc.y0 + (float)(bb.c0[1] + b) * gc.hy;
            const float wx = x - vc.src[0], wy = y - vc.src[1];
            const float n = wx * vc.cs + wy * vc.sn, d = wy * vc.cs - wx * vc.sn;
            const float ri = rcp(d);
            corner[t] = make_float2(n * ri, ri);
        }
        if (staged) {
            // element t -> (row, col) by a float reciprocal: exact for
            // t < 2^13, since (t + 1/2)/bw stays >= 1/(2 bw) from an integer
            const float ibw = 1.0f / (float)bw;
            int t0 = tid;
            asm volatile("" : "+v"(t0));
            for (int t = t0; t < bw * bh; t += 256) {
                const int row = (int)(((float)t + 0.5f) * ibw);
                const int col = t - row * bw;
                const long long pix = (long long)(bj0 + row) * nu + (bi0 + col);
                const PixelRay g = raysk[pix];
                float ginv[3];
                ray_inv(g, ginv);
                // first sample of the ray in the brick (a float estimate:
                // it only picks which segment origin to prepare)
                float tin = -3.0e38f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float t0 = (blo[a] - vc.Q[a]) * ginv[a];
                    const float t1 = (bhi[a] - vc.Q[a]) * ginv[a];
                    tin = fmaxf(tin, fminf(t0, t1));
                }
                const int sb = max(clamp_to_int(floor_t(tin)), 0) & ~(SEG - 1);
                const SegOrigin o = seg_origin(vc.Qd, g.D, sb);
                StagedRange er;
                StagedWalk ew;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float inv = ginv[a];
                    const float m = __builtin_fmaf(
                        4e-6f * (fabsf(vc.Q[a]) + cmax[a] + 1.0f), fabsf(inv), 1e-3f);
                    er.inv[a] = inv;
                    er.lo[a] = fminf(0.0f, inv) - m;
                }
                {
                    // the z layer's bounds, as a cell of the layer would
                    // compute them (cq = cz0 - Q_z in float)
                    const float inv = ginv[2];
                    const float t0 = (blo[2] - vc.Q[2]) * inv, t1 = t0 + inv;
                    const float m = __builtin_fmaf(
                        4e-6f * (fabsf(vc.Q[2]) + cmax[2] + 1.0f), fabsf(inv), 1e-3f);
                    er.zlo = fminf(t0, t1) - m;
                    er.zhi = fmaxf(t0, t1) + m;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ew.I[a] = (short)o.I[a];
                    ew.f[a] = o.f[a];
                    ew.Df[a] = (float)g.D[a];
                }
                // 32767 marks "no staged origin" (the plan bounds real
                // sample indices below 32767 * SEG)
                ew.sq = (short)min(sb / SEG, 32767);
                ew.r = (float)rk[pix];
                table[t].rg = er;
                table[t].wk = ew;
            }
        }
        __syncthreads();
        if (!valid) continue;
        // the cell's detector rectangle from its four xy corners (u) and
        // the extreme depths at its z faces (v), as box_footprint does
        const int cc = (cy - bb.c0[1]) * (CB_X + 1) + (cx - bb.c0[0]);
        const float2 k00 = corner[cc], k10 = corner[cc + 1];
        const float2 k01 = corner[cc + CB_X + 1], k11 = corner[cc + CB_X + 2];
        const float umin = dc.sdd * fminf(fminf(k00.x, k10.x), fminf(k01.x, k11.x));
        const float umax = dc.sdd * fmaxf(fmaxf(k00.x, k10.x), fmaxf(k01.x, k11.x));
        const float ia = fmaxf(fmaxf(k00.y, k10.y), fmaxf(k01.y, k11.y));  // 1 / nearest
        const float ib = fminf(fminf(k00.y, k10.y), fminf(k01.y, k11.y));  // 1 / farthest
        const float v0 = za * ia, v1 = za * ib, v2 = zb * ia, v3 = zb * ib;
        const float vmin = dc.sdd * fminf(fminf(v0, v1), fminf(v2, v3));
        const float vmax = dc.sdd * fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
        int i0, i1, j0, j1;
        pixel_range(dc, nu, nv, umin, umax, vmin, vmax, i0, i1, j0, j1);
        // the cell lies in the brick: keep its pixels inside the brick's
        // rectangle (they differ at most by rounding, inside the margin)
        i0 = max(i0, bi0);
        i1 = min(i1, bi1);
        j0 = max(j0, bj0);
        j1 = min(j1, bj1);
        const float Qf[3] = {vc.Q[0], vc.Q[1], vc.Q[2]};
        const CellRange cr = cell_range(Qf, cxf, cyf, czf);
        // 1 + 2 K_a of the staged margins (x, y)
        const float kw[2] = {1.0f + 8e-6f * (fabsf(vc.Q[0]) + cmax[0] + 1.0f),
                             1.0f + 8e-6f * (fabsf(vc.Q[1]) + cmax[1] + 1.0f)};
        // One flat loop over the cell's rectangle (nearly its exact
        // footprint): lanes with rectangles of different shapes then
        // diverge only in the total pixel count.
        const int w = i1 - i0 + 1, h = j1 - j0 + 1;
        const int npix = (w > 0 && h > 0) ? w * h : 0;
        int i = i0, j = j0;
        if constexpr (sizeof(T) == 4) {
            if (staged) {
                // the entry of pixel (i, j): a pointer advanced along the
                // rectangle (no per-visit multiplications)
                const StagedEntry *pe = table + (j0 - bj0) * bw + (i0 - bi0);
                const int skip = bw - w;  // from a row's end to the next row's start
                if (npix > 0) {
                    for (;;) {
                        const RayRef ray{raysk, nu, i, j};
                        visit_staged(acc, cr.cq, kw, *pe, ray, vc.Qd, cx, cy, cz);
                        ++pe;
                        if (++i > i1) {
                            if (++j > j1) break;
                            i = i0;
                            pe += skip;
                        }
                    }
                }
                continue;
            }
        }
        for (int q = 0; q < npix; ++q) {
            const RayRef ray{raysk, nu, i, j};
            const long long pix = (long long)j * nu + i;
            if (++i > i1) {
                i = i0;
                ++j;
            }
            visit_global<T>(acc, cr, ray, rk[pix], vc.Qd, cx, cy, cz);
        }
    }
    if (!valid) return;
    // The cell's index is formed again from the launch coordinates (passed
    // through an empty asm statement so the compiler does not keep the
    // first computation alive across the view loop, where it would spill).
    int b = (int)blockIdx.x, t = tid;
    asm volatile("" : "+v"(t), "+s"(b));
    const int br = xcd_tile(b, nb);
    const int ox = (br % nbx) * CB_X + t % CB_X;                       // cx + 1
    const int oy = ((br / nbx) % nby) * CB_Y + (t / CB_X) % CB_Y;      // cy + 1
    const int oz = (br / (nbx * nby)) * CB_Z + t / (CB_X * CB_Y);      // cz + 1
    const long long cp = cell_pitch(gc.nx);
    const long long ncell = cp * (gc.ny + 1) * (gc.nz + 1);
    const long long lin = (long long)ox + cp * (oy + (long long)(gc.ny + 1) * oz);
    T out[8];
    if constexpr (sizeof(T) == 4) {
        moments_to_corners(acc, out);
    } else {
#pragma unroll
        for (int o = 0; o < 8; ++o) out[o] = acc[o];
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) cells[o * ncell + lin] = out[o] * step;
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
    const long long cxn = cell_pitch(gc.nx), cxyn = cxn * (gc.ny + 1);
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

// The paper's Eq. (2) gradient, voxel-driven: one lane per voxel sums over
// the views L^3/(L0 l^2) times the bilinear interpolant of the residual at
// the voxel's imager point (zero beyond the outermost pixel centres), and
// scales by hx hy hz / (au av) (the transpose's scale).  The imager point
// in double (1/d from a float reciprocal refined by one double Newton
// step), the distance l and the interpolation in float, the sum in double.
// L^3/(L0 l^2)
// is evaluated as L0^2 l / d^3 (L/l = L0/d along the ray, d the depth of
// the voxel along the central ray).
constexpr int Q_BX = 64, Q_BY = 4;

__global__ __launch_bounds__(256) void k_eq2(const ViewConst *__restrict__ views, DetConst dc,
                                             GridConst gc, double hx, double hy, double hz,
                                             int nu, int nv, int nviews,
                                             const float *__restrict__ r,
                                             const float *__restrict__ f, double scale,
                                             double tau, float *__restrict__ out) {
    const int i = blockIdx.x * Q_BX + threadIdx.x;
    const int j = blockIdx.y * Q_BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= gc.nx || j >= gc.ny) return;
    const double sdd = dc.sddd, sdd2 = dc.sdd2d;
    const double iau = 1.0 / dc.aud, iav = 1.0 / dc.avd;
    const double ci = -dc.u0d * iau, cj = -dc.v0d * iav;  // index of u = 0, v = 0
    double sum = 0.0;
    for (int t = 0; t < nviews; ++t) {
        const ViewConst vc = views[t];
        // source-to-voxel vector in mm (index coordinates of the voxel
        // centre minus those of the source, times the spacing)
        const double wx = ((double)i - vc.Qd[0]) * hx;
        const double wy = ((double)j - vc.Qd[1]) * hy;
        const double wz = ((double)k - vc.Qd[2]) * hz;
        const double n = wx * vc.csd + wy * vc.snd;      // along e_u
        const double d = wy * vc.csd - wx * vc.snd;      // along e_w (depth)
        // 1/d from the float reciprocal and one Newton step in double: the
        // relative error squares, from ~2e-7 to ~4e-14
        const double id0 = (double)__builtin_amdgcn_rcpf((float)d);
        const double id = id0 * __builtin_fma(-d, id0, 2.0);
        const double fi = sdd * n * id * iau + ci;       // fractional pixel indices
        const double fj = sdd * wz * id * iav + cj;
        // l enters only the weight, where float's 1e-7 is ample
        const double l = (double)__builtin_sqrtf((float)(wx * wx + wy * wy + wz * wz));
        const double w = sdd2 * l * (id * id * id);
        const double i0d = __builtin_floor(fi), j0d = __builtin_floor(fj);
        const float a = (float)(fi - i0d), b = (float)(fj - j0d);
        const int i0 = (int)fmax(fmin(i0d, (double)nu), -2.0);
        const int j0 = (int)fmax(fmin(j0d, (double)nv), -2.0);
        const float *rt = r + (long long)t * nu * nv;
        const bool in0 = i0 >= 0 && i0 < nu, in1 = i0 + 1 >= 0 && i0 + 1 < nu;
        const bool jn0 = j0 >= 0 && j0 < nv, jn1 = j0 + 1 >= 0 && j0 + 1 < nv;
        const float r00 = (in0 && jn0) ? rt[(long long)j0 * nu + i0] : 0.0f;
        const float r10 = (in1 && jn0) ? rt[(long long)j0 * nu + i0 + 1] : 0.0f;
        const float r01 = (in0 && jn1) ? rt[(long long)(j0 + 1) * nu + i0] : 0.0f;
        const float r11 = (in1 && jn1) ? rt[(long long)(j0 + 1) * nu + i0 + 1] : 0.0f;
        const float v0 = r00 + a * (r10 - r00), v1 = r01 + a * (r11 - r01);
        sum += w * (double)(v0 + b * (v1 - v0));
    }
    const long long v = (long long)i + (long long)gc.nx * (j + (long long)gc.ny * k);
    const double s = scale * sum;
    out[v] = f ? (float)((double)f[v] - tau * s) : (float)s;
}

}  // namespace

namespace {

dim3 brick_grid(const cbct_geom &g) {
    return dim3((g.nx + 1 + CB_X - 1) / CB_X, (g.ny + 1 + CB_Y - 1) / CB_Y,
                (g.nz + 1 + CB_Z - 1) / CB_Z);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Geometry tables of the transpose: the ray table at offset 0, then the
// brick rectangles.
struct GeomLayout {
    size_t rects, total;  // byte offsets
};

GeomLayout geom_layout(const cbct_geom &g) {
    const dim3 b = brick_grid(g);
    GeomLayout l;
    l.rects = align256(sizeof(PixelRay) * (size_t)g.n_views * g.nu * g.nv);
    l.total = l.rects + sizeof(int4) * (size_t)b.x * b.y * b.z * g.n_views;
    return l;
}

}  // namespace

size_t bp_cells_bytes(const cbct_geom &g, size_t elem) {
    return align256(elem * 8 * (size_t)cell_pitch(g.nx) * (g.ny + 1) * (g.nz + 1));
}

size_t bp_geom_bytes(const cbct_geom &g) { return geom_layout(g).total; }

size_t bp_workspace_bytes(const cbct_geom &g, size_t elem) {
    return bp_cells_bytes(g, elem) + bp_geom_bytes(g);
}

void *bp_geom_in(void *ws, const cbct_geom &g, size_t elem) {
    return (char *)ws + bp_cells_bytes(g, elem);
}

void cell_pass_config(int32_t out[4]) {
    out[0] = CB_X;
    out[1] = CB_Y;
    out[2] = CB_Z;
    out[3] = TABLE;
}

hipError_t launch_bp_prepare(const cbct_plan &p, void *geom, hipStream_t s) {
    const GeomLayout l = geom_layout(p.g);
    char *base = (char *)geom;
    hipLaunchKernelGGL(k_rays, dim3((p.g.nu + 63) / 64, (p.g.nv + 3) / 4, p.g.n_views), dim3(256),
                       0, s, p.d_views, p.det, p.g.nu, p.g.nv, (PixelRay *)base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 b = brick_grid(p.g);
    const long long n = (long long)b.x * b.y * b.z * p.g.n_views;
    hipLaunchKernelGGL(k_brick_rects, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       p.d_views, p.det, p.grid, p.g.nu, p.g.nv, (int)b.x, (int)b.y, (int)b.z,
                       p.g.n_views, (int4 *)(base + l.rects));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backproject_cells(const cbct_plan &p, const T *r, void *cells,
                                    const void *geom, hipStream_t s) {
    const GeomLayout l = geom_layout(p.g);
    const char *base = (const char *)geom;
    const dim3 b = brick_grid(p.g);
    hipLaunchKernelGGL(k_cells<T>, dim3(b.x * b.y * b.z), dim3(256), 0, s, p.d_views, p.det, p.grid,
                       p.g.nu, p.g.nv, p.g.n_views, (const PixelRay *)base,
                       (const int4 *)(base + l.rects), r, (T *)cells, (T)p.g.step);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_cells(const cbct_plan &p, const void *ws, const T *f, double tau,
                               T *out, hipStream_t s) {
    dim3 grid((p.g.nx + G_BX - 1) / G_BX, (p.g.ny + G_BY - 1) / G_BY, p.g.nz);
    hipLaunchKernelGGL(k_gather<T>, grid, dim3(G_BX, G_BY), 0, s, p.grid, (const T *)ws, f,
                       (T)tau, out);
    return hipGetLastError();
}

hipError_t launch_eq2(const cbct_plan &p, const float *r, const float *f, double tau,
                      float *out, hipStream_t s) {
    const double scale = p.g.hx * p.g.hy * p.g.hz / (p.g.au * p.g.av);
    dim3 grid((p.g.nx + Q_BX - 1) / Q_BX, (p.g.ny + Q_BY - 1) / Q_BY, p.g.nz);
    hipLaunchKernelGGL(k_eq2, grid, dim3(Q_BX, Q_BY), 0, s, p.d_views, p.det, p.grid, p.g.hx,
                       p.g.hy, p.g.hz, p.g.nu, p.g.nv, p.g.n_views, r, f, scale, tau, out);
    return hipGetLastError();
}

template hipError_t launch_backproject_cells<float>(const cbct_plan &, const float *, void *,
                                                    const void *, hipStream_t);
template hipError_t launch_backproject_cells<double>(const cbct_plan &, const double *, void *,
                                                     const void *, hipStream_t);
template hipError_t launch_gather_cells<float>(const cbct_plan &, const void *, const float *,
                                               double, float *, hipStream_t);
template hipError_t launch_gather_cells<double>(const cbct_plan &, const void *,
                                                const double *, double, double *, hipStream_t);

}  // namespace cbct
