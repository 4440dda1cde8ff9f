// Forward cone-beam projection P (Eq. (1)): ray-driven trilinear ray march.
//
// One lane per ray; a wavefront covers 64 neighbouring detector columns of
// one row, so at equal sample index the 64 lanes touch neighbouring voxels
// and the eight trilinear taps of the wave share cache lines.  The volume is
// read from a copy with a one-voxel zero border, so every tap of every
// sample the ray takes is in bounds without per-sample tests: the sample
// interval is computed exactly (cell of every sample in [-1, N-1]).
#include "ray.hpp"

namespace cbct {

namespace {

constexpr int PROJ_BX = 64;
constexpr int PROJ_BY = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_pad(const T *__restrict__ f, T *__restrict__ fp,
                                             int nx, int ny, int nz) {
    const int px = nx + 2, py = ny + 2, pz = nz + 2;
    const long long total = (long long)px * py * pz;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(t % px);
        const long long r = t / px;
        const int j = (int)(r % py);
        const int k = (int)(r / py);
        T v = T(0);
        if (i >= 1 && i <= nx && j >= 1 && j <= ny && k >= 1 && k <= nz)
            v = f[(i - 1) + (long long)nx * ((j - 1) + (long long)ny * (k - 1))];
        fp[t] = v;
    }
}

// True if sample n of the ray lies in a cell with index in [-1, N-1] on
// every axis, i.e. q in [-1, N).
template <typename T>
__device__ __forceinline__ bool in_box(int n, const T Q[3], const T D[3], const GridConst &gc) {
    const T nf = (T)n;
    const T q0 = sample_coord(nf, D[0], Q[0]);
    const T q1 = sample_coord(nf, D[1], Q[1]);
    const T q2 = sample_coord(nf, D[2], Q[2]);
    return q0 >= T(-1) && q0 < T(gc.nx) && q1 >= T(-1) && q1 < T(gc.ny) && q2 >= T(-1) &&
           q2 < T(gc.nz);
}

// Exact sample interval [n0, n1] of a ray (empty if n0 > n1).
template <typename T>
__device__ __forceinline__ void ray_interval(const T Q[3], const T D[3], const GridConst &gc,
                                             int &n0, int &n1) {
    T lo = T(-1e30), hi = T(1e30), a = T(0), b = T(0);
    bool ok = axis_interval(Q[0], D[0], T(-1), T(gc.nx), a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    ok = ok && axis_interval(Q[1], D[1], T(-1), T(gc.ny), a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    ok = ok && axis_interval(Q[2], D[2], T(-1), T(gc.nz), a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    if (!ok || lo > hi + T(2)) {
        n0 = 1;
        n1 = 0;
        return;
    }
    n0 = clamp_to_int(floor_t(lo));
    n1 = clamp_to_int(floor_t(hi)) + 1;
    if (n0 < 0) n0 = 0;
    // shrink to the exact interval, then grow in case the estimate was short
    while (n0 <= n1 && !in_box(n0, Q, D, gc)) ++n0;
    while (n1 >= n0 && !in_box(n1, Q, D, gc)) --n1;
    if (n0 <= n1) {
        while (n0 > 0 && in_box(n0 - 1, Q, D, gc)) --n0;
        while (in_box(n1 + 1, Q, D, gc)) ++n1;
    }
}

// Block-wide sum of one double per thread into partials[block].
__device__ __forceinline__ void block_sum_store(double v, double *partials, int block_lin) {
    __shared__ double red[8];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wid = tid >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w];
        partials[block_lin] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_project(const ViewConst *__restrict__ views, DetConst dc,
                                                 GridConst gc, int nu, int nv,
                                                 const T *__restrict__ fp,
                                                 const T *__restrict__ Y, T *__restrict__ out,
                                                 double *__restrict__ partials, T step) {
    const int i = blockIdx.x * PROJ_BX + threadIdx.x;
    const int j = blockIdx.y * PROJ_BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool valid = i < nu && j < nv;
    const ViewConst vc = views[k];
    double Q[3], D[3];
    ray_setup(vc, dc, valid ? i : 0, valid ? j : 0, Q, D);
    int n0 = 1, n1 = 0;
    if (valid) ray_interval(Q, D, gc, n0, n1);
    const int px = gc.nx + 2;
    const int pxy = px * (gc.ny + 2);
    double acc = 0.0;
    double nf = (double)n0;
    for (int n = n0; n <= n1; ++n, nf += 1.0) {
        const double q0 = sample_coord(nf, D[0], Q[0]);
        const double q1 = sample_coord(nf, D[1], Q[1]);
        const double q2 = sample_coord(nf, D[2], Q[2]);
        const double f0 = floor_t(q0), f1 = floor_t(q1), f2 = floor_t(q2);
        const T wx = (T)(q0 - f0), wy = (T)(q1 - f1), wz = (T)(q2 - f2);
        const int base = ((int)f2 + 1) * pxy + ((int)f1 + 1) * px + ((int)f0 + 1);
        const T *p = fp + base;
        const T c000 = p[0], c100 = p[1], c010 = p[px], c110 = p[px + 1];
        const T c001 = p[pxy], c101 = p[pxy + 1], c011 = p[pxy + px], c111 = p[pxy + px + 1];
        const T c00 = c000 + wx * (c100 - c000);
        const T c10 = c010 + wx * (c110 - c010);
        const T c01 = c001 + wx * (c101 - c001);
        const T c11 = c011 + wx * (c111 - c011);
        const T c0 = c00 + wy * (c10 - c00);
        const T c1 = c01 + wy * (c11 - c01);
        acc += (double)(c0 + wz * (c1 - c0));
    }
    double sq = 0.0;
    if (valid) {
        const long long idx = ((long long)k * nv + j) * nu + i;
        T val = (T)(acc * (double)step);
        if (Y) val -= Y[idx];
        out[idx] = val;
        sq = (double)val * (double)val;
    }
    if (partials) {
        const int blin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum_store(sq, partials, blin);
    }
}

__global__ __launch_bounds__(256) void k_count(const ViewConst *__restrict__ views, DetConst dc,
                                               GridConst gc, int nu, int nv,
                                               unsigned long long *count) {
    const int i = blockIdx.x * PROJ_BX + threadIdx.x;
    const int j = blockIdx.y * PROJ_BY + threadIdx.y;
    const int k = blockIdx.z;
    unsigned long long c = 0;
    if (i < nu && j < nv) {
        double Q[3], D[3];
        ray_setup(views[k], dc, i, j, Q, D);
        int n0, n1;
        ray_interval(Q, D, gc, n0, n1);
        if (n1 >= n0) c = (unsigned long long)(n1 - n0 + 1);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(count, c);
}

dim3 project_grid(const cbct_plan &p) {
    return dim3((p.g.nu + PROJ_BX - 1) / PROJ_BX, (p.g.nv + PROJ_BY - 1) / PROJ_BY, p.g.n_views);
}

}  // namespace

size_t project_partials_count(const cbct_plan &p) {
    dim3 g = project_grid(p);
    return (size_t)g.x * g.y * g.z;
}

template <typename T>
hipError_t launch_pad(const cbct_plan &p, const T *f, T *fpad, hipStream_t s) {
    const long long total = (long long)(p.g.nx + 2) * (p.g.ny + 2) * (p.g.nz + 2);
    long long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_pad<T>, dim3((unsigned)blocks), dim3(256), 0, s, f, fpad, p.g.nx,
                       p.g.ny, p.g.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const cbct_plan &p, const T *fpad, const T *Y, T *out,
                          double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_project<T>, project_grid(p), dim3(PROJ_BX, PROJ_BY), 0, s, p.d_views,
                       p.det, p.grid, p.g.nu, p.g.nv, fpad, Y, out, partials, (T)p.g.step);
    return hipGetLastError();
}

hipError_t launch_count_samples(const cbct_plan &p, unsigned long long *count, hipStream_t s) {
    hipLaunchKernelGGL(k_count, project_grid(p), dim3(PROJ_BX, PROJ_BY), 0, s, p.d_views, p.det,
                       p.grid, p.g.nu, p.g.nv, count);
    return hipGetLastError();
}

template hipError_t launch_pad<float>(const cbct_plan &, const float *, float *, hipStream_t);
template hipError_t launch_pad<double>(const cbct_plan &, const double *, double *, hipStream_t);
template hipError_t launch_project<float>(const cbct_plan &, const float *, const float *,
                                          float *, double *, hipStream_t);
template hipError_t launch_project<double>(const cbct_plan &, const double *, const double *,
                                           double *, double *, hipStream_t);

}  // namespace cbct
