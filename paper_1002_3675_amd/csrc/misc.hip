// Small kernels of the solver: reductions, fills, and the multigrid
// transfers (2x2 detector binning, 2x2x2 restriction, trilinear
// prolongation at cell-centred fine voxels).
#include "cbct_internal.hpp"

namespace cbct {

namespace {

__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ x, long long n,
                                               double *__restrict__ partials) {
    double s = 0.0;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
         t += (long long)gridDim.x * 256) {
        const double v = x[t];
        s += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Partial sums of (a - b)^2 and a^2 per block, in double, fixed order.
__global__ __launch_bounds__(256) void k_diff_sums(const float *__restrict__ a,
                                                   const float *__restrict__ b, long long n,
                                                   double *__restrict__ partials) {
    double d = 0.0, m = 0.0;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
         t += (long long)gridDim.x * 256) {
        const double x = a[t], e = x - (double)b[t];
        d += e * e;
        m += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        d += __shfl_down(d, off, 64);
        m += __shfl_down(m, off, 64);
    }
    __shared__ double red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = d;
        red[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partials[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// out[c] = sum_i partials[i * ncols + c], one block, fixed order per lane.
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partials, int n,
                                                int ncols, double *__restrict__ out) {
    for (int c = 0; c < ncols; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) s += partials[(long long)i * ncols + c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        __shared__ double red[4];
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_fill(float *__restrict__ x, long long n, float v) {
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
         t += (long long)gridDim.x * 256)
        x[t] = v;
}

// out = x / sqrt(*denom)  (denominator is a device sum of squares)
__global__ __launch_bounds__(256) void k_scale(const float *__restrict__ x, long long n,
                                               const double *__restrict__ sumsq,
                                               float *__restrict__ out) {
    const double inv = 1.0 / __builtin_sqrt(*sumsq);
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
         t += (long long)gridDim.x * 256)
        out[t] = (float)((double)x[t] * inv);
}

__global__ __launch_bounds__(256) void k_bin(const float *__restrict__ y, int nu, int nv,
                                             long long total, float *__restrict__ out) {
    const int cu = nu / 2, cv = nv / 2;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const int i = (int)(t % cu);
        const long long r = t / cu;
        const int j = (int)(r % cv);
        const long long k = r / cv;
        const float *b = y + (k * nv + 2 * j) * (long long)nu + 2 * i;
        out[t] = 0.25f * ((b[0] + b[1]) + (b[nu] + b[nu + 1]));
    }
}

__global__ __launch_bounds__(256) void k_restrict(const float *__restrict__ f, int nx, int ny,
                                                  long long total, float *__restrict__ out) {
    const int cx = nx / 2, cy = ny / 2;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const int i = (int)(t % cx);
        const long long r = t / cx;
        const int j = (int)(r % cy);
        const long long k = r / cy;
        const float *b = f + ((2 * k) * ny + 2 * j) * (long long)nx + 2 * i;
        const long long sz = (long long)nx * ny;
        const float s = ((b[0] + b[1]) + (b[nx] + b[nx + 1])) +
                        ((b[sz] + b[sz + 1]) + (b[sz + nx] + b[sz + nx + 1]));
        out[t] = 0.125f * s;
    }
}

// Coarse coordinate of fine index i: (i + 1/2)/2 - 1/2 clamped to [0, n-1];
// returns base index and weight of the upper neighbour.
__device__ __forceinline__ void prolong_axis(int i, int n, int &c0, float &w) {
    float c = 0.5f * (float)i - 0.25f;
    c = fminf(fmaxf(c, 0.0f), (float)(n - 1));
    int b = (int)floorf(c);
    if (b > n - 2) b = n - 2;
    if (b < 0) b = 0;
    c0 = b;
    w = n > 1 ? c - (float)b : 0.0f;
}

__global__ __launch_bounds__(256) void k_prolong(const float *__restrict__ fc, int cx, int cy,
                                                 int cz, float *__restrict__ ff, int nx, int ny,
                                                 long long total) {
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const int i = (int)(t % nx);
        const long long r = t / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        int bx, by, bz;
        float wx, wy, wz;
        prolong_axis(i, cx, bx, wx);
        prolong_axis(j, cy, by, wy);
        prolong_axis(k, cz, bz, wz);
        const int dx = cx > 1 ? 1 : 0, dy = cy > 1 ? cx : 0;
        const long long dz = cz > 1 ? (long long)cx * cy : 0;
        const float *p = fc + bx + (long long)cx * (by + (long long)cy * bz);
        const float c00 = p[0] + wx * (p[dx] - p[0]);
        const float c10 = p[dy] + wx * (p[dy + dx] - p[dy]);
        const float c01 = p[dz] + wx * (p[dz + dx] - p[dz]);
        const float c11 = p[dz + dy] + wx * (p[dz + dy + dx] - p[dz + dy]);
        const float c0 = c00 + wy * (c10 - c00);
        const float c1 = c01 + wy * (c11 - c01);
        ff[t] = c0 + wz * (c1 - c0);
    }
}

unsigned grid_for(long long n) {
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_sumsq(const float *x, size_t n, double *partials, int *n_partials,
                        hipStream_t s) {
    unsigned b = grid_for((long long)n);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_sumsq, dim3(b), dim3(256), 0, s, x, (long long)n, partials);
    *n_partials = (int)b;
    return hipGetLastError();
}

hipError_t launch_diff_sums(const float *a, const float *b, size_t n, double *partials,
                            int *n_partials, hipStream_t s) {
    unsigned nb = grid_for((long long)n);
    if (nb > (unsigned)DIFF_BLOCKS) nb = DIFF_BLOCKS;
    hipLaunchKernelGGL(k_diff_sums, dim3(nb), dim3(256), 0, s, a, b, (long long)n, partials);
    *n_partials = (int)nb;
    return hipGetLastError();
}

hipError_t launch_reduce_sum(const double *partials, int n, double *out, int ncols,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, n, ncols, out);
    return hipGetLastError();
}

// Independent FMA chains per lane; the sum is stored so the chains stay live.
__device__ __forceinline__ float fma_t(float x, float a, float b) { return __builtin_fmaf(x, a, b); }
__device__ __forceinline__ double fma_t(double x, double a, double b) { return __builtin_fma(x, a, b); }

template <typename T>
__global__ __launch_bounds__(256) void k_probe_fma(T *__restrict__ out, int iters, T a, T b) {
    T x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (T)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = fma_t(x[c], a, b);
    }
    T sum = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) sum += x[c];
    out[(long long)blockIdx.x * 256 + threadIdx.x] = sum;
}

// flop of one probe launch: blocks x 256 lanes x iters x 8 chains x 2
hipError_t launch_probe_fma(bool fp64, void *out, int blocks, int iters, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(k_probe_fma<double>, dim3(blocks), dim3(256), 0, s, (double *)out,
                           iters, 0.999, 0.001);
    else
        hipLaunchKernelGGL(k_probe_fma<float>, dim3(blocks), dim3(256), 0, s, (float *)out,
                           iters, 0.999f, 0.001f);
    return hipGetLastError();
}

// y = ln(ref / max(c, min_count)), ref = flat[i] or i0; double arithmetic.
__global__ __launch_bounds__(256) void k_log_counts(const float *__restrict__ counts,
                                                    const float *__restrict__ flat, double i0,
                                                    double min_count, float *y, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double c = fmax((double)counts[i], min_count);
    const double ref = flat ? (double)flat[i] : i0;
    y[i] = (float)log(ref / c);
}

hipError_t launch_log_counts(const float *counts, const float *flat, double i0,
                             double min_count, float *y, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_log_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, counts,
                       flat, i0, min_count, y, n);
    return hipGetLastError();
}

hipError_t launch_fill(float *x, size_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for((long long)n)), dim3(256), 0, s, x, (long long)n, v);
    return hipGetLastError();
}

hipError_t launch_scale(const float *x, size_t n, const double *denom, float *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(grid_for((long long)n)), dim3(256), 0, s, x, (long long)n,
                       denom, out);
    return hipGetLastError();
}

hipError_t launch_bin_detector(const float *y, int nu, int nv, int nviews, float *out,
                               hipStream_t s) {
    const long long total = (long long)nviews * (nv / 2) * (nu / 2);
    hipLaunchKernelGGL(k_bin, dim3(grid_for(total)), dim3(256), 0, s, y, nu, nv, total, out);
    return hipGetLastError();
}

hipError_t launch_restrict(const float *f, int nx, int ny, int nz, float *out, hipStream_t s) {
    const long long total = (long long)(nx / 2) * (ny / 2) * (nz / 2);
    hipLaunchKernelGGL(k_restrict, dim3(grid_for(total)), dim3(256), 0, s, f, nx, ny, total, out);
    return hipGetLastError();
}

hipError_t launch_prolong(const float *fc, int cx, int cy, int cz, float *ff, int nx, int ny,
                          int nz, hipStream_t s) {
    const long long total = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_prolong, dim3(grid_for(total)), dim3(256), 0, s, fc, cx, cy, cz, ff, nx,
                       ny, total);
    return hipGetLastError();
}

}  // namespace cbct
