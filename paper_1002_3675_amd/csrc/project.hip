// Forward cone-beam projection P (Eq. (1)): ray-driven trilinear ray march.
//
// One lane per ray; a wavefront covers 64 neighbouring detector columns of
// one row, so at equal sample index the 64 lanes touch neighbouring voxels
// and the eight trilinear taps of the wave share cache lines.  The volume is
// read from a copy with a one-voxel zero border, so every tap of every
// sample the ray takes is in bounds without per-sample tests: the sample
// interval is computed exactly (cell of every sample in [-1, N-1]).  Float
// volumes are read with raw buffer loads (32-bit offsets, x-neighbour pairs
// as one 8-byte load; the descriptor's range returns zero past the end).
#include "ray.hpp"

namespace cbct {

namespace {

constexpr int PROJ_BX = 64;
constexpr int PROJ_BY = 4;

// Zero-bordered copies of f: fp is [nz+2][ny+2][nx+2] (x fastest) and, when
// fpt is not NULL, fpt is [nz+2][nx+2][ny+2] (y fastest).  Views whose rays
// run mostly along x read fpt, so that the 64 lanes of a wavefront (64
// neighbouring rays, spread across the rays' direction) still touch
// consecutive addresses.  The transposed copy is written through a 32x32
// LDS tile per xy slab so both copies are written with coalesced rows.
template <typename T>
__global__ __launch_bounds__(256) void k_pad(const T *__restrict__ f, T *__restrict__ fp,
                                             T *__restrict__ fpt, int nx, int ny, int nz) {
    __shared__ T tile[32][33];
    const int px = nx + 2, py = ny + 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32, k = blockIdx.z;  // padded coords
    const bool kin = k >= 1 && k <= nz;
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + tx, j = j0 + r;
        T v = T(0);
        if (kin && i >= 1 && i <= nx && j >= 1 && j <= ny)
            v = f[(i - 1) + (long long)nx * ((j - 1) + (long long)ny * (k - 1))];
        if (i < px && j < py) fp[i + (long long)px * (j + (long long)py * k)] = v;
        tile[r][tx] = v;
    }
    if (!fpt) return;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + tx, i = i0 + r;  // y fastest
        if (i < px && j < py) fpt[j + (long long)py * (i + (long long)px * k)] = tile[tx][r];
    }
}

// Cell of sample n (the definition shared with the transpose).
template <typename T>
__device__ __forceinline__ void sample_cell(const double Q[3], const double D[3],
                                            const float Df[3], int n, int c[3]) {
    if constexpr (sizeof(T) == 4) {
        const int ns = n & ~(SEG - 1);
        const SegOrigin o = seg_origin(Q, D, ns);
        const float m = (float)(n - ns);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int dc;
            float w;
            seg_axis(m, Df[a], o.f[a], dc, w);
            c[a] = o.I[a] + dc;
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            c[a] = (int)floor_t(sample_coord((double)n, D[a], Q[a]));
    }
}

// True if sample n lies in a cell with index in [-1, N-1] on every axis.
template <typename T>
__device__ __forceinline__ bool in_box(int n, const double Q[3], const double D[3],
                                       const float Df[3], const GridConst &gc) {
    int c[3];
    sample_cell<T>(Q, D, Df, n, c);
    return c[0] >= -1 && c[0] < gc.nx && c[1] >= -1 && c[1] < gc.ny && c[2] >= -1 &&
           c[2] < gc.nz;
}

// Exact sample interval [n0, n1] of a ray (empty if n0 > n1).  The estimate
// from the double ray is widened by one sample and then moved to the exact
// ends with the shared cell definition; cells are monotone in n along each
// axis, so the in-box samples form one interval.
template <typename T>
__device__ __forceinline__ void ray_interval(const double Q[3], const double D[3],
                                             const float Df[3], const GridConst &gc, int &n0,
                                             int &n1) {
    double lo = -1e30, hi = 1e30, a = 0.0, b = 0.0;
    bool ok = axis_interval(Q[0], D[0], -1.0, (double)gc.nx, a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    ok = ok && axis_interval(Q[1], D[1], -1.0, (double)gc.ny, a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    ok = ok && axis_interval(Q[2], D[2], -1.0, (double)gc.nz, a, b);
    lo = a > lo ? a : lo;
    hi = b < hi ? b : hi;
    if (!ok || lo > hi + 2.0) {
        n0 = 1;
        n1 = 0;
        return;
    }
    n0 = clamp_to_int(floor_t(lo));
    n1 = clamp_to_int(floor_t(hi)) + 1;
    if (n0 < 0) n0 = 0;
    while (n0 <= n1 && !in_box<T>(n0, Q, D, Df, gc)) ++n0;
    while (n1 >= n0 && !in_box<T>(n1, Q, D, Df, gc)) --n1;
    if (n0 <= n1) {
        while (n0 > 0 && in_box<T>(n0 - 1, Q, D, Df, gc)) --n0;
        while (in_box<T>(n1 + 1, Q, D, Df, gc)) ++n1;
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

// Two adjacent floats at byte offset voff + soff (soff wave-uniform); the
// backend merges the two loads into one dwordx2.
__device__ __forceinline__ float2 load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const unsigned a = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    const unsigned b = __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4, soff, 0);
    return make_float2(__builtin_bit_cast(float, a), __builtin_bit_cast(float, b));
}

__device__ __forceinline__ int wave_min(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Ray sum over [n0, n1] for float volumes: segment origins in double, the
// per-sample cell and weights in float.  All lanes of the wavefront step
// through the same sample index n (the union of their intervals, each lane
// masked outside its own), so at every step the 64 neighbouring rays sit
// at the same distance from the source and their taps share cache lines;
// the loop bounds are wave-uniform.
__device__ __forceinline__ double march_float(const double Q[3], const double D[3],
                                              const float Df[3], int n0, int n1,
                                              __amdgpu_buffer_rsrc_t vol, int px, int pxy) {
    double acc = 0.0;
    const bool any = n0 <= n1;
    const int wlo = wave_min(any ? n0 : 0x7fffffff);
    const int whi = wave_max(any ? n1 : -1);
    for (int s = wlo & ~(SEG - 1); s <= whi; s += SEG) {
        const SegOrigin o = seg_origin(Q, D, s);
        const int base = (o.I[2] + 1) * pxy + (o.I[1] + 1) * px + (o.I[0] + 1);
        const int ma = (wlo > s ? wlo : s) - s;
        const int mb = (whi < s + SEG - 1 ? whi : s + SEG - 1) - s;
        float seg = 0.0f;
        float m = (float)ma;
        for (int mi = ma; mi <= mb; ++mi, m += 1.0f) {
            const int n = s + mi;
            if (n < n0 || n > n1) continue;
            int dx, dy, dz;
            float wx, wy, wz;
            seg_axis(m, Df[0], o.f[0], dx, wx);
            seg_axis(m, Df[1], o.f[1], dy, wy);
            seg_axis(m, Df[2], o.f[2], dz, wz);
            const int off = 4 * (base + dx + __mul24(dy, px) + __mul24(dz, pxy));
            const float2 a0 = load_pair(vol, off, 0);
            const float2 a1 = load_pair(vol, off, 4 * px);
            const float2 b0 = load_pair(vol, off, 4 * pxy);
            const float2 b1 = load_pair(vol, off, 4 * (pxy + px));
            const float c00 = a0.x + wx * (a0.y - a0.x);
            const float c10 = a1.x + wx * (a1.y - a1.x);
            const float c01 = b0.x + wx * (b0.y - b0.x);
            const float c11 = b1.x + wx * (b1.y - b1.x);
            const float c0 = c00 + wy * (c10 - c00);
            const float c1 = c01 + wy * (c11 - c01);
            seg += c0 + wz * (c1 - c0);
        }
        acc += (double)seg;
    }
    return acc;
}

// Ray sum for double volumes: double coordinates per sample.
__device__ __forceinline__ double march_double(const double Q[3], const double D[3], int n0,
                                               int n1, const double *__restrict__ fp, int px,
                                               int pxy) {
    double acc = 0.0;
    double nf = (double)n0;
    for (int n = n0; n <= n1; ++n, nf += 1.0) {
        const double q0 = sample_coord(nf, D[0], Q[0]);
        const double q1 = sample_coord(nf, D[1], Q[1]);
        const double q2 = sample_coord(nf, D[2], Q[2]);
        const double f0 = floor_t(q0), f1 = floor_t(q1), f2 = floor_t(q2);
        const double wx = q0 - f0, wy = q1 - f1, wz = q2 - f2;
        const int base = ((int)f2 + 1) * pxy + ((int)f1 + 1) * px + ((int)f0 + 1);
        const double *p = fp + base;
        const double c00 = p[0] + wx * (p[1] - p[0]);
        const double c10 = p[px] + wx * (p[px + 1] - p[px]);
        const double c01 = p[pxy] + wx * (p[pxy + 1] - p[pxy]);
        const double c11 = p[pxy + px] + wx * (p[pxy + px + 1] - p[pxy + px]);
        const double c0 = c00 + wy * (c10 - c00);
        const double c1 = c01 + wy * (c11 - c01);
        acc += c0 + wz * (c1 - c0);
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_project(const ViewConst *__restrict__ views, DetConst dc,
                                                 GridConst gc, int nu, int nv,
                                                 const T *__restrict__ fp,
                                                 const T *__restrict__ fpt, int fp_elems,
                                                 const T *__restrict__ Y, T *__restrict__ out,
                                                 double *__restrict__ partials, T step) {
    const int i = blockIdx.x * PROJ_BX + threadIdx.x;
    const int j = blockIdx.y * PROJ_BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool valid = i < nu && j < nv;
    const ViewConst vc = views[k];
    double Q[3], D[3];
    float Df[3];
    ray_setup(vc, dc, valid ? i : 0, valid ? j : 0, Q, D);
    // rays mostly along x: march the y-fastest copy with x and y exchanged
    // (the per-axis cell arithmetic is unchanged by the relabelling)
    const bool swap = fpt != nullptr && fabsf(vc.sn) > fabsf(vc.cs);
    if (swap) {
        double t = Q[0];
        Q[0] = Q[1];
        Q[1] = t;
        t = D[0];
        D[0] = D[1];
        D[1] = t;
        const int ti = gc.nx;
        gc.nx = gc.ny;
        gc.ny = ti;
    }
    to_float3(D, Df);
    int n0 = 1, n1 = 0;
    if (valid) ray_interval<T>(Q, D, Df, gc, n0, n1);
    const int px = gc.nx + 2;
    const int pxy = px * (gc.ny + 2);
    double acc;
    if constexpr (sizeof(T) == 4) {
        const __amdgpu_buffer_rsrc_t vol = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(swap ? fpt : fp), (short)0, fp_elems * 4, 0x00020000);
        acc = march_float(Q, D, Df, n0, n1, vol, px, pxy);
    } else {
        acc = march_double(Q, D, n0, n1, fp, px, pxy);
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
        float Df[3];
        ray_setup(views[k], dc, i, j, Q, D);
        to_float3(D, Df);
        int n0, n1;
        ray_interval<float>(Q, D, Df, gc, n0, n1);
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

size_t padded_count(const cbct_plan &p) {
    return (size_t)(p.g.nx + 2) * (p.g.ny + 2) * (p.g.nz + 2);
}

// fpad holds padded_count elements for the x-fastest copy; float volumes
// get the y-fastest copy right after it (2 * padded_count in total).
size_t pad_buffer_count(const cbct_plan &p, size_t elem_size) {
    return elem_size == 4 ? 2 * padded_count(p) : padded_count(p);
}

template <typename T>
hipError_t launch_pad(const cbct_plan &p, const T *f, T *fpad, hipStream_t s) {
    dim3 grid((p.g.nx + 2 + 31) / 32, (p.g.ny + 2 + 31) / 32, p.g.nz + 2);
    T *fpt = sizeof(T) == 4 ? fpad + padded_count(p) : nullptr;
    hipLaunchKernelGGL(k_pad<T>, grid, dim3(256), 0, s, f, fpad, fpt, p.g.nx, p.g.ny, p.g.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const cbct_plan &p, const T *fpad, const T *Y, T *out,
                          double *partials, hipStream_t s) {
    const long long elems = (long long)padded_count(p);
    const T *fpt = sizeof(T) == 4 ? fpad + elems : nullptr;
    hipLaunchKernelGGL(k_project<T>, project_grid(p), dim3(PROJ_BX, PROJ_BY), 0, s, p.d_views,
                       p.det, p.grid, p.g.nu, p.g.nv, fpad, fpt, (int)elems, Y, out, partials,
                       (T)p.g.step);
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
