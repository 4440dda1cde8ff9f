// TV pieces of Algorithm A1: the projected gradient step of Step 2/3 and
// the E1 energy of Eq. (1).
//
// D_a z = (z[v + e_a] - z[v]) / h_a (zero at the last index of axis a) and
// D^T p = sum_a ([i_a > 0] p_a[v - e_a] - [i_a < N_a - 1] p_a[v]) / h_a.
// The update at v needs p = Dz/|Dz|_eps at v and at v - e_a, i.e. z at v,
// its six face neighbours and the six points v - e_a + e_b.  The sweep is
// HBM-bound (12 bytes per voxel: read z and g, write z); a wavefront covers
// 64 consecutive x so every neighbour load is a coalesced row.
#include "cbct_internal.hpp"

namespace cbct {

namespace {

constexpr int TV_BX = 64;
constexpr int TV_BY = 4;

struct TvArgs {
    int nx, ny, nz;
    float ihx, ihy, ihz;  // 1/h
    float eps2;
};

// p = D z / |D z|_eps at (i, j, k), all in-bounds indices.
__device__ __forceinline__ void normalised_grad(const float *__restrict__ z, const TvArgs &a, int i,
                                                int j, int k, long long v, float &px, float &py,
                                                float &pz) {
    const long long sx = 1, sy = a.nx, sz = (long long)a.nx * a.ny;
    const float zc = z[v];
    const float gx = (i < a.nx - 1) ? (z[v + sx] - zc) * a.ihx : 0.0f;
    const float gy = (j < a.ny - 1) ? (z[v + sy] - zc) * a.ihy : 0.0f;
    const float gz = (k < a.nz - 1) ? (z[v + sz] - zc) * a.ihz : 0.0f;
    const float inv = __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + a.eps2);
    px = gx * inv;
    py = gy * inv;
    pz = gz * inv;
}

__global__ __launch_bounds__(256) void k_tv_sweep(TvArgs a, const float *__restrict__ z,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ out, float beta, float step,
                                                  int nonneg) {
    const int i = blockIdx.x * TV_BX + threadIdx.x;
    const int j = blockIdx.y * TV_BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const long long sy = a.nx, sz = (long long)a.nx * a.ny;
    const long long v = i + sy * j + sz * k;
    float px, py, pz;
    normalised_grad(z, a, i, j, k, v, px, py, pz);
    float div = 0.0f;
    if (i < a.nx - 1) div -= px * a.ihx;
    if (j < a.ny - 1) div -= py * a.ihy;
    if (k < a.nz - 1) div -= pz * a.ihz;
    if (i > 0) {
        float qx, qy, qz;
        normalised_grad(z, a, i - 1, j, k, v - 1, qx, qy, qz);
        div += qx * a.ihx;
    }
    if (j > 0) {
        float qx, qy, qz;
        normalised_grad(z, a, i, j - 1, k, v - sy, qx, qy, qz);
        div += qy * a.ihy;
    }
    if (k > 0) {
        float qx, qy, qz;
        normalised_grad(z, a, i, j, k - 1, v - sz, qx, qy, qz);
        div += qz * a.ihz;
    }
    const float zc = z[v];
    float zn = zc - step * (div + beta * (zc - g[v]));
    if (nonneg) zn = fmaxf(zn, 0.0f);
    out[v] = zn;
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
    return a;
}

dim3 tv_grid(const GridConst &gc) {
    return dim3((gc.nx + TV_BX - 1) / TV_BX, (gc.ny + TV_BY - 1) / TV_BY, gc.nz);
}

}  // namespace

hipError_t launch_tv_sweep(const GridConst &gc, const float *z, const float *g, float *out,
                           float beta, float eps, float step, int nonneg, hipStream_t s) {
    hipLaunchKernelGGL(k_tv_sweep, tv_grid(gc), dim3(TV_BX, TV_BY), 0, s, args_of(gc, eps), z, g,
                       out, beta, step, nonneg);
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
