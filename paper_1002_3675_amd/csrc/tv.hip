// TV pieces of Algorithm A1: the projected gradient step of Step 2/3 and
// the E1 energy of Eq. (1).
//
// D_a z = (z[v + e_a] - z[v]) / h_a (zero at the last index of axis a) and
// D^T p = sum_a ([i_a > 0] p_a[v - e_a] - [i_a < N_a - 1] p_a[v]) / h_a.
// The update at v needs p = Dz/|Dz|_eps at v and at v - e_a.  The sweep is
// HBM-bound (12 bytes per voxel: read z and g, write z).  A workgroup owns a
// 32 x 8 column of voxels and marches a chunk of z planes: each plane of z
// (with a one-voxel halo) is staged once in LDS, p is computed once per
// position of the tile and its low halo, and p_z of the plane below stays
// in a register, so every voxel costs one read of z and g, one write, and
// one reciprocal square root.  Arrays whose rows are a multiple of 4 voxels
// and 16-byte aligned take k_tv_sweep4 (one wavefront per tile, four voxels
// per lane, 16-byte loads and stores); others take the 256-lane k_tv_sweep.
#include "cbct_internal.hpp"

namespace cbct {

namespace {

constexpr int TV_BX = 64;
constexpr int TV_BY = 4;
constexpr int ST_X = 32, ST_Y = 8;  // sweep tile
constexpr int ST_Z = 16;            // longest z chunk
// A sweep should put at least this many workgroups in flight (8 per CU):
// grids with few 32 x 8 columns get shorter z chunks.
constexpr int SWEEP_MIN_GROUPS = 2048;

struct TvArgs {
    int nx, ny, nz;
    float ihx, ihy, ihz;  // 1/h
    float eps2;
    int zc;  // z chunk of the sweep (planes)
};

// Tiles of a sweep: 32 x 8 columns of the xy plane (x-fastest, then y) in
// chunks of a.zc planes, chunk-major in launch order.  Within a chunk each
// XCD takes one contiguous range of columns (xcd_tile), so neighbouring
// tiles share their halo lines in one L2.  The remap stays inside a chunk:
// over the whole grid it would hand the last, shorter chunks to one XCD.
struct SweepTile {
    int i0, j0, k0, k1;
};

__device__ __forceinline__ SweepTile sweep_tile(const TvArgs &a, int b) {
    const int ntx = (a.nx + ST_X - 1) / ST_X, nty = (a.ny + ST_Y - 1) / ST_Y;
    const int tpc = ntx * nty;  // tiles per chunk
    const int bz = b / tpc;
    const int tin = xcd_tile(b - bz * tpc, tpc);
    const int bx = tin % ntx, by = tin / ntx;
    SweepTile t;
    t.i0 = bx * ST_X;
    t.j0 = by * ST_Y;
    t.k0 = bz * a.zc;
    t.k1 = min(t.k0 + a.zc, a.nz);
    return t;
}

// One projected gradient step on a 32 x 8 tile marching a chunk of planes.
// Plane k + 2 is fetched into registers while plane k is processed.
__global__ __launch_bounds__(256) void k_tv_sweep(TvArgs a, const float *__restrict__ z,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ out, float beta, float step,
                                                  int nonneg) {
    // z planes k and k+1 with a one-voxel halo on every side of the tile
    __shared__ float zs[2][ST_Y + 2][ST_X + 2];
    // p = Dz/|Dz|_eps of plane k at the tile and its low halo
    __shared__ float ps[3][ST_Y + 1][ST_X + 1];
    const int tid = threadIdx.x;
    const int tx = tid & (ST_X - 1), ty = tid / ST_X;
    const SweepTile st = sweep_tile(a, blockIdx.x);
    const int i0 = st.i0, j0 = st.j0, k0 = st.k0, k1 = st.k1;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < a.nx && j < a.ny;
    const long long sy = a.nx, sz = (long long)a.nx * a.ny;

    // plane elements of this lane: t = tid and t = tid + 256 of the
    // (ST_Y + 2) x (ST_X + 2) halo tile
    constexpr int NP = (ST_Y + 2) * (ST_X + 2);
    int off[2];
    bool inb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int t = tid + 256 * e;
        const int jj = t / (ST_X + 2), ii = t % (ST_X + 2);
        const int gi = i0 - 1 + ii, gj = j0 - 1 + jj;
        inb[e] = t < NP && gi >= 0 && gi < a.nx && gj >= 0 && gj < a.ny;
        off[e] = inb[e] ? gi + a.nx * gj : 0;
    }
    auto fetch = [&](int k, float r[2]) {
#pragma unroll
        for (int e = 0; e < 2; ++e) r[e] = (inb[e] && k < a.nz) ? z[off[e] + sz * k] : 0.0f;
    };
    auto put = [&](int slot, const float r[2]) {
        float *zp = &zs[slot][0][0];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (tid + 256 * e < NP) zp[tid + 256 * e] = r[e];
    };

    // p_z of the plane below the chunk, for this lane's voxel
    float pz_prev = 0.0f;
    if (own && k0 > 0) {
        const long long v = i + sy * j + sz * (k0 - 1);
        const float zc = z[v];
        const float gx = (i < a.nx - 1) ? (z[v + 1] - zc) * a.ihx : 0.0f;
        const float gy = (j < a.ny - 1) ? (z[v + sy] - zc) * a.ihy : 0.0f;
        const float gz = (z[v + sz] - zc) * a.ihz;  // k0 - 1 < nz - 1
        pz_prev = gz * __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
    }
    float nxt[2];
    fetch(k0, nxt);
    put(k0 & 1, nxt);
    fetch(k0 + 1, nxt);
    for (int k = k0; k < k1; ++k) {
        const int A = k & 1, B = A ^ 1;
        put(B, nxt);                       // plane k + 1
        if (k + 2 < k1 + 1) fetch(k + 2, nxt);  // in flight during this plane
        const long long v = i + sy * j + sz * k;
        const float gv = own ? g[v] : 0.0f;
        __syncthreads();
        for (int t = tid; t < (ST_Y + 1) * (ST_X + 1); t += 256) {
            const int jj = t / (ST_X + 1), ii = t % (ST_X + 1);
            const int gi = i0 - 1 + ii, gj = j0 - 1 + jj;
            const float zc = zs[A][jj][ii];
            const float gx = (gi < a.nx - 1) ? (zs[A][jj][ii + 1] - zc) * a.ihx : 0.0f;
            const float gy = (gj < a.ny - 1) ? (zs[A][jj + 1][ii] - zc) * a.ihy : 0.0f;
            const float gz = (k < a.nz - 1) ? (zs[B][jj][ii] - zc) * a.ihz : 0.0f;
            const float inv = __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
            ps[0][jj][ii] = gx * inv;
            ps[1][jj][ii] = gy * inv;
            ps[2][jj][ii] = gz * inv;
        }
        const float zc = zs[A][ty + 1][tx + 1];
        __syncthreads();
        if (own) {
            const float pz = ps[2][ty + 1][tx + 1];
            float div = 0.0f;
            if (i < a.nx - 1) div -= ps[0][ty + 1][tx + 1] * a.ihx;
            if (j < a.ny - 1) div -= ps[1][ty + 1][tx + 1] * a.ihy;
            if (k < a.nz - 1) div -= pz * a.ihz;
            if (i > 0) div += ps[0][ty + 1][tx] * a.ihx;
            if (j > 0) div += ps[1][ty][tx + 1] * a.ihy;
            if (k > 0) div += pz_prev * a.ihz;
            float zn = zc - step * (div + beta * (zc - gv));
            if (nonneg) zn = fmaxf(zn, 0.0f);
            out[v] = zn;
            pz_prev = pz;
        }
    }
}

// The same step with 16-byte accesses: one wavefront per 32 x 8 tile, each
// lane owning four consecutive x voxels of one row (nx a multiple of 4,
// arrays 16-byte aligned).  z planes are staged in LDS with float4 loads
// (plus the two x-halo columns), g is read and the result written as
// float4, and the barriers are those of a single wavefront.  The
// arithmetic per voxel is that of k_tv_sweep, in the same order.
constexpr int W_X = 32, W_Y = 8;  // tile
constexpr int W_PITCH = 40;       // LDS row: column 3 is x = i0 - 1, 4..35 the tile, 36 x = i0 + 32

__global__ __launch_bounds__(64) void k_tv_sweep4(TvArgs a, const float *__restrict__ z,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ out, float beta, float step,
                                                  int nonneg) {
    // z planes k and k+1: rows y = j0 - 1 .. j0 + 8
    __shared__ __attribute__((aligned(16))) float zs[2][W_Y + 2][W_PITCH];
    // p_x and p_y of plane k: rows y = j0 - 1 .. j0 + 7, columns as zs
    __shared__ __attribute__((aligned(16))) float ps[2][W_Y + 1][W_PITCH];
    const int lane = threadIdx.x;
    const int tx = lane & 7, ty = lane >> 3;
    const SweepTile st = sweep_tile(a, blockIdx.x);
    const int i0 = st.i0, j0 = st.j0, k0 = st.k0, k1 = st.k1;
    const int i = i0 + 4 * tx, j = j0 + ty;  // this lane's first voxel
    const bool own = i < a.nx && j < a.ny;   // all four, since 4 | nx
    const long long sy = a.nx, sz = (long long)a.nx * a.ny;

    // staging work of this lane: interior float4 (row r1 = ty, and for
    // lanes 0..15 also row 8 + lane / 8), or for lanes 16..35 one x-halo
    // element (row (lane - 16) / 2, column low or high)
    const int rB = lane < 16 ? 8 + (lane >> 3) : -1;           // second interior row
    const int hrow = (lane >= 16 && lane < 36) ? (lane - 16) >> 1 : -1;
    const int hcol = (lane & 1) ? 36 : 3;                        // LDS column of the halo
    const int hx = (lane & 1) ? i0 + W_X : i0 - 1;               // its x
    auto row_ok = [&](int r) {
        const int y = j0 - 1 + r;
        return r >= 0 && y >= 0 && y < a.ny;
    };
    const bool qA = i < a.nx && row_ok(ty);
    const bool qB = rB >= 0 && i < a.nx && row_ok(rB);
    const bool qH = hrow >= 0 && hx >= 0 && hx < a.nx && row_ok(hrow);
    const long long oA = (long long)i + sy * (j0 - 1 + ty);
    const long long oB = (long long)i + sy * (j0 - 1 + rB);
    const long long oH = (long long)hx + sy * (j0 - 1 + hrow);
    struct Plane {
        float4 A, B;
        float H;
    };
    auto fetch = [&](int k, Plane &pl) {
        const bool kin = k < a.nz;
        pl.A = (kin && qA) ? *(const float4 *)(z + oA + sz * k) : make_float4(0.f, 0.f, 0.f, 0.f);
        pl.B = (kin && qB) ? *(const float4 *)(z + oB + sz * k) : make_float4(0.f, 0.f, 0.f, 0.f);
        pl.H = (kin && qH) ? z[oH + sz * k] : 0.0f;
    };
    auto put = [&](int slot, const Plane &pl) {
        *(float4 *)&zs[slot][ty][4 + 4 * tx] = pl.A;
        if (rB >= 0) *(float4 *)&zs[slot][rB][4 + 4 * tx] = pl.B;
        if (hrow >= 0) zs[slot][hrow][hcol] = pl.H;
    };

    // p_z of the plane below the chunk, for this lane's voxels
    float pz_prev[4] = {0.f, 0.f, 0.f, 0.f};
    if (own && k0 > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const long long v = i + q + sy * j + sz * (k0 - 1);
            const float zc = z[v];
            const float gx = (i + q < a.nx - 1) ? (z[v + 1] - zc) * a.ihx : 0.0f;
            const float gy = (j < a.ny - 1) ? (z[v + sy] - zc) * a.ihy : 0.0f;
            const float gz = (z[v + sz] - zc) * a.ihz;  // k0 - 1 < nz - 1
            pz_prev[q] = gz * __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
        }
    }
    Plane nxt;
    fetch(k0, nxt);
    put(k0 & 1, nxt);
    fetch(k0 + 1, nxt);
    // the lane's extra p position: low x column (x = i0 - 1, 9 rows) for
    // lanes 0..8, low y row (y = j0 - 1, 32 columns) for lanes 9..40
    const int ex_r = lane < 9 ? lane : (lane < 41 ? 0 : -1);
    const int ex_c = lane < 9 ? 3 : 4 + (lane - 9);
    const int ex_x = i0 - 1 + (ex_c - 3), ex_y = j0 - 1 + ex_r;
    for (int k = k0; k < k1; ++k) {
        const int A = k & 1, B = A ^ 1;
        put(B, nxt);                             // plane k + 1
        if (k + 2 < k1 + 1) fetch(k + 2, nxt);  // in flight during this plane
        const long long v = i + sy * j + sz * k;
        const float4 gv = own ? *(const float4 *)(g + v) : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        // p at the lane's own four positions (row ty + 1 of ps)
        const int r = ty + 1, c = 4 + 4 * tx;
        const float4 zc4 = *(const float4 *)&zs[A][r][c];
        const float zr = zs[A][r][c + 4];
        const float4 zu4 = *(const float4 *)&zs[A][r + 1][c];
        const float4 zn4 = *(const float4 *)&zs[B][r][c];
        const float zcv[4] = {zc4.x, zc4.y, zc4.z, zc4.w};
        const float zxn[4] = {zc4.y, zc4.z, zc4.w, zr};
        const float zyn[4] = {zu4.x, zu4.y, zu4.z, zu4.w};
        const float zzn[4] = {zn4.x, zn4.y, zn4.z, zn4.w};
        float px[4], py[4], pz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float gx = (i + q < a.nx - 1) ? (zxn[q] - zcv[q]) * a.ihx : 0.0f;
            const float gy = (j < a.ny - 1) ? (zyn[q] - zcv[q]) * a.ihy : 0.0f;
            const float gz = (k < a.nz - 1) ? (zzn[q] - zcv[q]) * a.ihz : 0.0f;
            const float inv = __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
            px[q] = gx * inv;
            py[q] = gy * inv;
            pz[q] = gz * inv;
        }
        *(float4 *)&ps[0][r][c] = make_float4(px[0], px[1], px[2], px[3]);
        *(float4 *)&ps[1][r][c] = make_float4(py[0], py[1], py[2], py[3]);
        if (ex_r >= 0) {
            // p at the low halo position (only p_x or p_y is read there)
            const float zc = zs[A][ex_r][ex_c];
            const float gx = (ex_x < a.nx - 1) ? (zs[A][ex_r][ex_c + 1] - zc) * a.ihx : 0.0f;
            const float gy = (ex_y < a.ny - 1) ? (zs[A][ex_r + 1][ex_c] - zc) * a.ihy : 0.0f;
            const float gz = (k < a.nz - 1) ? (zs[B][ex_r][ex_c] - zc) * a.ihz : 0.0f;
            const float inv = __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
            ps[0][ex_r][ex_c] = gx * inv;
            ps[1][ex_r][ex_c] = gy * inv;
        }
        __syncthreads();
        if (own) {
            const float4 pl = *(const float4 *)&ps[0][r][c - 4];  // columns c - 4 .. c - 1
            const float4 pu = *(const float4 *)&ps[1][r - 1][c];
            const float pxm[4] = {pl.w, px[0], px[1], px[2]};
            const float pym[4] = {pu.x, pu.y, pu.z, pu.w};
            const float gvv[4] = {gv.x, gv.y, gv.z, gv.w};
            float res[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float div = 0.0f;
                if (i + q < a.nx - 1) div -= px[q] * a.ihx;
                if (j < a.ny - 1) div -= py[q] * a.ihy;
                if (k < a.nz - 1) div -= pz[q] * a.ihz;
                if (i + q > 0) div += pxm[q] * a.ihx;
                if (j > 0) div += pym[q] * a.ihy;
                if (k > 0) div += pz_prev[q] * a.ihz;
                float zn = zcv[q] - step * (div + beta * (zcv[q] - gvv[q]));
                if (nonneg) zn = fmaxf(zn, 0.0f);
                res[q] = zn;
                pz_prev[q] = pz[q];
            }
            *(float4 *)(out + v) = make_float4(res[0], res[1], res[2], res[3]);
        }
    }
}

// Per-block partial sums of |Dz| and sqrt(|Dz|^2 + eps^2), in double.
__global__ __launch_bounds__(256) void k_tv_energy(TvArgs a, const float *__restrict__ z,
                                                   double eps2, double *__restrict__ partials) {
    const int i = blockIdx.x * TV_BX + threadIdx.x;
    const int j = blockIdx.y * TV_BY + threadIdx.y;
    const int k = blockIdx.z;
    double s0 = 0.0, s1 = 0.0;
    if (i < a.nx && j < a.ny) {
        const long long sy = a.nx, sz = (long long)a.nx * a.ny;
        const long long v = i + sy * j + sz * k;
        const double zc = z[v];
        const double hx = a.ihx, hy = a.ihy, hz = a.ihz;
        const double gx = (i < a.nx - 1) ? ((double)z[v + 1] - zc) * hx : 0.0;
        const double gy = (j < a.ny - 1) ? ((double)z[v + sy] - zc) * hy : 0.0;
        const double gz = (k < a.nz - 1) ? ((double)z[v + sz] - zc) * hz : 0.0;
        const double m2 = gx * gx + gy * gy + gz * gz;
        s0 = __builtin_sqrt(m2);
        s1 = __builtin_sqrt(m2 + eps2);
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off, 64);
        s1 += __shfl_down(s1, off, 64);
    }
    __shared__ double red[2][4];
    const int tid = threadIdx.x + TV_BX * threadIdx.y;
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s0;
        red[1][tid >> 6] = s1;
    }
    __syncthreads();
    if (tid == 0) {
        const int blin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partials[2 * blin] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partials[2 * blin + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

TvArgs args_of(const GridConst &gc, double eps) {
    TvArgs a;
    a.nx = gc.nx;
    a.ny = gc.ny;
    a.nz = gc.nz;
    a.ihx = (float)(1.0 / (double)gc.hx);
    a.ihy = (float)(1.0 / (double)gc.hy);
    a.ihz = (float)(1.0 / (double)gc.hz);
    a.eps2 = (float)(eps * eps);
    // z chunk: up to ST_Z planes, shorter when the columns alone would
    // leave the CUs short of workgroups (each chunk re-reads the plane
    // below it and one above: (zc + 2) / zc of the z reads)
    const int cols = ((gc.nx + ST_X - 1) / ST_X) * ((gc.ny + ST_Y - 1) / ST_Y);
    const int want = (SWEEP_MIN_GROUPS + cols - 1) / cols;  // chunks wanted
    int zc = (gc.nz + want - 1) / want;
    zc = zc < 2 ? 2 : (zc > ST_Z ? ST_Z : zc);
    a.zc = zc;
    return a;
}

dim3 tv_grid(const GridConst &gc) {
    return dim3((gc.nx + TV_BX - 1) / TV_BX, (gc.ny + TV_BY - 1) / TV_BY, gc.nz);
}

}  // namespace

hipError_t launch_tv_sweep(const GridConst &gc, const float *z, const float *g, float *out,
                           float beta, float eps, float step, int nonneg, hipStream_t s) {
    const TvArgs a = args_of(gc, eps);
    const int grid = ((gc.nx + ST_X - 1) / ST_X) * ((gc.ny + ST_Y - 1) / ST_Y) *
                     ((gc.nz + a.zc - 1) / a.zc);
    const bool vec4 = gc.nx % 4 == 0 && ((uintptr_t)z | (uintptr_t)g | (uintptr_t)out) % 16 == 0;
    static_assert(W_X == ST_X && W_Y == ST_Y, "both sweeps use the same tiles");
    if (vec4)
        hipLaunchKernelGGL(k_tv_sweep4, dim3(grid), dim3(64), 0, s, a, z, g, out, beta, step,
                           nonneg);
    else
        hipLaunchKernelGGL(k_tv_sweep, dim3(grid), dim3(256), 0, s, a, z, g, out, beta, step,
                           nonneg);
    return hipGetLastError();
}

size_t tv_energy_partials_count(const GridConst &gc) {
    dim3 g = tv_grid(gc);
    return (size_t)2 * g.x * g.y * g.z;
}

hipError_t launch_tv_energy(const GridConst &gc, const float *z, double eps, double *partials,
                            int *n_partials, hipStream_t s) {
    dim3 g = tv_grid(gc);
    hipLaunchKernelGGL(k_tv_energy, g, dim3(TV_BX, TV_BY), 0, s, args_of(gc, eps), z, eps * eps,
                       partials);
    *n_partials = (int)(g.x * g.y * g.z);
    return hipGetLastError();
}

}  // namespace cbct
