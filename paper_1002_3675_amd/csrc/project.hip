// Forward cone-beam projection P (Eq. (1)): ray-driven trilinear ray march.
//
// One lane per ray.  The float path (k_project_tile) gives a workgroup a
// square tile of neighbouring rays and stages the volume boxes they cross in
// LDS; the double path (k_project) lets a wavefront cover 64 neighbouring
// detector columns of one row, so at equal sample index the 64 lanes touch
// neighbouring voxels and the taps of the wave share cache lines.  The volume is
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

// Zero-bordered copy of f: fp is [nz+2][ny+2][nx+2] (x fastest).
template <typename T>
__global__ __launch_bounds__(256) void k_pad(const T *__restrict__ f, T *__restrict__ fp, int nx,
                                             int ny, int nz) {
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

// Sum of the trilinear samples m = ma .. mb of one chunk from the staged
// box (row pitch RX, plane pitch RXY floats, base the LDS offset of the
// segment origin's cell): seg_axis's coordinates and weights, the LDS offset
// of the floors formed in float (exact: |offset| < 2^24), m counted in float
// (exact below 2^24); two samples per loop step, summed in order.  RXC > 0
// fixes the row pitch at compile time.
template <int RXC>
__device__ __forceinline__ float staged_samples(const float *vol, int base, int RXr, int RXY,
                                                float m, float mb, const float Df[3],
                                                const float of[3]) {
    const int RX = RXC > 0 ? RXC : RXr;
    const float RXf = (float)RX, RXYf = (float)RXY;
    float seg = 0.0f;
    auto sample = [&](float m) {
        const float lx = __builtin_fmaf(m, Df[0], of[0]);
        const float ly = __builtin_fmaf(m, Df[1], of[1]);
        const float lz = __builtin_fmaf(m, Df[2], of[2]);
        const float fx = __builtin_floorf(lx), fy = __builtin_floorf(ly),
                    fz = __builtin_floorf(lz);
        const float wx = lx - fx, wy = ly - fy, wz = lz - fz;
        const float *p = vol + base + (int)__builtin_fmaf(fz, RXYf, __builtin_fmaf(fy, RXf, fx));
        const float *q = p + RXY;
        const float c00 = p[0] + wx * (p[1] - p[0]);
        const float c10 = p[RX] + wx * (p[RX + 1] - p[RX]);
        const float c01 = q[0] + wx * (q[1] - q[0]);
        const float c11 = q[RX] + wx * (q[RX + 1] - q[RX]);
        const float c0 = c00 + wy * (c10 - c00);
        const float c1 = c01 + wy * (c11 - c01);
        seg += c0 + wz * (c1 - c0);
    };
    for (; m + 1.0f <= mb; m += 2.0f) {
        sample(m);
        sample(m + 1.0f);
    }
    if (m <= mb) sample(m);
    return seg;
}

// ---------------------------------------------------------------------------
// Float projector with LDS-staged volume.  A workgroup owns a 16 x 16 tile of
// detector pixels of one view; its 256 rays advance together through chunks
// of consecutive sample indices.  The indices are cut into pieces of
// TILE_SUB; for each piece the four corner rays of the tile bound (with a
// margin for the curvature of the ray bundle) the box of cells every sample
// of the piece can touch.  The boxes of up to BOX_TAB pieces are computed
// together, one piece per lane, and then grouped into chunks, one aligned
// block of TILE_MERGE pieces per lane: a chunk is a run of pieces of one
// block whose boxes' bounding box fits TILE_LDS floats, or a run of pieces
// whose own boxes do not fit.  A fitting chunk's box of the zero-bordered
// volume is loaded straight into LDS (buffer loads to LDS, one z plane at a
// time) and the eight trilinear taps of every sample are read from LDS; an
// unfitting chunk reads its taps from global memory.  The samples, their
// cells and weights are exactly those of sample_cell and seg_axis (the
// definitions the transpose shares), whatever the chunking.  A square tile
// keeps the bundle, and so the box, narrow in both detector directions.
// Where a tile spans many cells (pixels near the voxel size) single pieces
// still fit; where it spans few, runs spread the per-chunk staging and
// segment-origin work over more samples.
constexpr int TILE_U = 16, TILE_V = 16;
constexpr int TILE_SUB = 16;    // samples per box
constexpr int TILE_MERGE = 8;   // boxes per chunk at most
constexpr int TILE_LDS = 5632;  // floats (larger boxes stage more slowly than they save)
constexpr int BOX_TAB = 128;    // boxes computed together
static_assert(SEG % (TILE_SUB * TILE_MERGE) == 0, "a block of pieces lies inside one segment");
static_assert(BOX_TAB % TILE_MERGE == 0 && BOX_TAB <= 256, "whole blocks per box table");
static_assert(TILE_LDS < (1 << 13), "the plane row division is exact below 2^13");

__device__ __forceinline__ void unpack_box(int4 e, int b0[3], int b1[3]) {
    const int pk[3] = {e.x, e.y, e.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b0[a] = (int)(short)(pk[a] & 0xffff);
        b1[a] = pk[a] >> 16;
    }
}

// Whether the box fits the LDS box with its odd row pitch.  No product
// overflows: grid dimensions are at most 32000, so every extent is below
// 2^15 and a plane below 2^30, and the box is formed only for a plane that
// fits.
__device__ __forceinline__ bool box_fits(const int b0[3], const int b1[3]) {
    const int RX = b1[0] - b0[0] + 1, RY = b1[1] - b0[1] + 1, RZ = b1[2] - b0[2] + 1;
    if (RX <= 0 || RY <= 0 || RZ <= 0) return false;
    const int npl = (RX | 1) * RY;
    return npl <= TILE_LDS && npl * RZ <= TILE_LDS;
}

// Groups the pieces [q0, q1) of one block of the table into chunks: the
// entry of a chunk's first piece takes the chunk's box and, in w, its
// length in pieces (negative for a chunk read from global memory).
__device__ __forceinline__ void group_block(int4 *tab, int q0, int q1) {
    for (int q = q0; q < q1;) {
        int b0[3], b1[3];
        unpack_box(tab[q], b0, b1);
        const bool fits = box_fits(b0, b1);
        int e = q + 1;
        for (; e < q1; ++e) {
            int u0[3], u1[3];
            unpack_box(tab[e], u0, u1);
            if (fits) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u0[a] = min(u0[a], b0[a]);
                    u1[a] = max(u1[a], b1[a]);
                }
                if (!box_fits(u0, u1)) break;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    b0[a] = u0[a];
                    b1[a] = u1[a];
                }
            } else if (box_fits(u0, u1)) {
                break;
            }
        }
        tab[q] = make_int4((b0[0] & 0xffff) | (b1[0] << 16), (b0[1] & 0xffff) | (b1[1] << 16),
                           (b0[2] & 0xffff) | (b1[2] << 16), fits ? e - q : q - e);
        q = e;
    }
}

// At most 80 VGPRs: six wavefronts per SIMD (six groups of 24 KB of LDS per
// CU) instead of the five that the unconstrained 95 allow.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_project_tile(
    const ViewConst *__restrict__ views, DetConst dc, GridConst gc, int nu, int nv,
    const float *__restrict__ fp, int fp_elems, const float *__restrict__ Y,
    float *__restrict__ out, double *__restrict__ partials, float step, int margin) {
    __shared__ float vol[TILE_LDS];
    __shared__ int4 boxes[BOX_TAB];  // piece boxes, packed b0 | b1 << 16 per axis
    __shared__ int red[2][4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    // tiles u-fastest, then v, then view; contiguous per XCD, so the rays
    // of neighbouring tiles stage overlapping bricks through one L2
    const int ntu = (nu + TILE_U - 1) / TILE_U, ntv = (nv + TILE_V - 1) / TILE_V;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tu = tile % ntu, tv = (tile / ntu) % ntv, k = tile / (ntu * ntv);
    const int i = tu * TILE_U + (tid & (TILE_U - 1));
    const int j = tv * TILE_V + tid / TILE_U;
    const bool valid = i < nu && j < nv;
    const ViewConst vc = views[k];
    double Q[3], D[3];
    float Df[3];
    ray_setup(vc, dc, valid ? i : 0, valid ? j : 0, Q, D);
    to_float3(D, Df);
    int n0 = 1, n1 = 0;
    if (valid) ray_interval<float>(Q, D, Df, gc, n0, n1);
    // union of the tile's sample intervals
    const bool any = n0 <= n1;
    int lo = wave_min(any ? n0 : 0x7fffffff), hi = wave_max(any ? n1 : -1);
    if (lane == 0) {
        red[0][wid] = lo;
        red[1][wid] = hi;
    }
    __syncthreads();
    lo = min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3]));
    hi = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
    const int N[3] = {gc.nx, gc.ny, gc.nz};
    const int px = gc.nx + 2, pxy = px * (gc.ny + 2);
    const __amdgpu_buffer_rsrc_t gvol =
        __builtin_amdgcn_make_buffer_rsrc((void *)fp, (short)0, fp_elems * 4, 0x00020000);
    double acc = 0.0;
    // piece c holds the sample indices nc0 + TILE_SUB c .. nc0 + TILE_SUB (c + 1) - 1;
    // blocks of pieces start at multiples of TILE_SUB * TILE_MERGE
    const int nc0 = lo & ~(TILE_SUB * TILE_MERGE - 1);
    const int npieces = hi >= nc0 ? (hi - nc0) / TILE_SUB + 1 : 0;
    for (int cg = 0; cg < npieces; cg += BOX_TAB) {
        __syncthreads();  // readers of the previous group's boxes are done
        if (tid < BOX_TAB && cg + tid < npieces) {
            // box of padded cells [b0, b1] per axis touched by piece cg + tid,
            // from the tile's four corner rays
            const int nc = nc0 + TILE_SUB * (cg + tid);
            const int ci0 = tu * TILE_U, ci1 = min(ci0 + TILE_U - 1, nu - 1);
            const int cj0 = tv * TILE_V, cj1 = min(cj0 + TILE_V - 1, nv - 1);
            double Dc[4][3], Qc[3];
            ray_setup(vc, dc, ci0, cj0, Qc, Dc[0]);
            ray_setup(vc, dc, ci1, cj0, Qc, Dc[1]);
            ray_setup(vc, dc, ci0, cj1, Qc, Dc[2]);
            ray_setup(vc, dc, ci1, cj1, Qc, Dc[3]);
            int pk[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double qmin = 1e300, qmax = -1e300;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double qa = Qc[a] + (double)nc * Dc[c][a];
                    const double qb = Qc[a] + (double)(nc + TILE_SUB - 1) * Dc[c][a];
                    qmin = fmin(qmin, fmin(qa, qb));
                    qmax = fmax(qmax, fmax(qa, qb));
                }
                // cells floor(q) in [-1, N-1] read padded indices cell+1 and
                // cell+2; an empty range keeps b0 > b1 after the clamps
                const int b0 = min(max((int)floor(fmax(qmin, -4.0)) - margin + 1, 0), N[a] + 2);
                const int b1 =
                    max(min((int)floor(fmin(qmax, (double)N[a] + 4.0)) + margin + 2, N[a] + 1), -1);
                pk[a] = (b0 & 0xffff) | (b1 << 16);
            }
            boxes[tid] = make_int4(pk[0], pk[1], pk[2], 0);
        }
        __syncthreads();
        const int cend = min(npieces, cg + BOX_TAB);
        if (tid < BOX_TAB / TILE_MERGE && cg + TILE_MERGE * tid < cend)
            group_block(boxes, TILE_MERGE * tid, min(TILE_MERGE * (tid + 1), cend - cg));
        __syncthreads();
        for (int c = cg; c < cend;) {
            const int nc = nc0 + TILE_SUB * c;
            const int4 ent = boxes[c - cg];
            // identical in every lane: kept in scalar registers
            int b0[3], b1[3];
            unpack_box(make_int4(__builtin_amdgcn_readfirstlane(ent.x),
                                 __builtin_amdgcn_readfirstlane(ent.y),
                                 __builtin_amdgcn_readfirstlane(ent.z), 0),
                       b0, b1);
            const int run = __builtin_amdgcn_readfirstlane(ent.w);
            const bool staged = run > 0;
            const int len = TILE_SUB * (staged ? run : -run);
            c += staged ? run : -run;
            const int RX = b1[0] - b0[0] + 1, RY = b1[1] - b0[1] + 1, RZ = b1[2] - b0[2] + 1;
            // LDS rows have an odd pitch, so rays spread across rows (views whose
            // rays run along x) do not pile onto one bank
            const int RXP = RX | 1;
            __syncthreads();  // the previous chunk's readers are done
            if (staged) {
                // Plane z of the box is RXP * RY consecutive LDS elements, x
                // fastest; each wavefront loads 64 consecutive elements
                // straight into LDS.  Element t of a plane is row t / RXP, by
                // a float reciprocal: exact for t < 2^13, since (t + 1/2)/RXP
                // stays >= 1/(2 RXP) from an integer and the reciprocal and
                // product err by under 2^-21 relative.
                const int npl = RXP * RY;
                const float ipx = __builtin_amdgcn_rcpf((float)RXP);
                for (int rz = 0; rz < RZ; ++rz) {
                    const int gpl = (b0[2] + rz) * pxy + b0[1] * px + b0[0];
                    for (int t0 = 64 * wid; t0 < npl; t0 += 256) {
                        const int t = t0 + lane;
                        if (t < npl) {
                            const int row = (int)(((float)t + 0.5f) * ipx);
                            const int x = t - __mul24(row, RXP);
                            // x = RX (the odd pitch's pad column, never read)
                            // loads a neighbour or, past the end, zero
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                gvol, (__attribute__((address_space(3))) void *)&vol[rz * npl + t0],
                                4, (gpl + __mul24(row, px) + x) * 4, 0, 0, 0);
                        }
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);  // the loads have landed in LDS
            }
            __syncthreads();
            const int na = max(n0, nc), nb = min(n1, nc + len - 1);
            if (na > nb) continue;
            const int s = nc & ~(SEG - 1);
            const SegOrigin o = seg_origin(Q, D, s);
            float seg = 0.0f;
            if (staged) {
                const int RXY = RXP * RY;
                const int base = (o.I[2] + 1 - b0[2]) * RXY + (o.I[1] + 1 - b0[1]) * RXP +
                                 (o.I[0] + 1 - b0[0]);
                const float ma = (float)(na - s), mb = (float)(nb - s);
                // common row pitches as constants: the row offsets then sit in
                // the LDS instructions' immediates
                switch (RXP) {
#define CBCT_PITCH(n)                                                                   \
    case n:                                                                             \
        seg = staged_samples<n>(vol, base, RXP, RXY, ma, mb, Df, o.f);                   \
        break;
                    CBCT_PITCH(5) CBCT_PITCH(7) CBCT_PITCH(9) CBCT_PITCH(11) CBCT_PITCH(13)
                    CBCT_PITCH(15) CBCT_PITCH(17) CBCT_PITCH(19) CBCT_PITCH(21) CBCT_PITCH(23)
                    CBCT_PITCH(25) CBCT_PITCH(27) CBCT_PITCH(29) CBCT_PITCH(31) CBCT_PITCH(33)
                    CBCT_PITCH(35) CBCT_PITCH(37) CBCT_PITCH(39) CBCT_PITCH(41)
#undef CBCT_PITCH
                    default:
                        seg = staged_samples<0>(vol, base, RXP, RXY, ma, mb, Df, o.f);
                }
            } else {
                const int base = (o.I[2] + 1) * pxy + (o.I[1] + 1) * px + (o.I[0] + 1);
                const float mb = (float)(nb - s);
                for (float m = (float)(na - s); m <= mb; m += 1.0f) {
                    int dx, dy, dz;
                    float wx, wy, wz;
                    seg_axis(m, Df[0], o.f[0], dx, wx);
                    seg_axis(m, Df[1], o.f[1], dy, wy);
                    seg_axis(m, Df[2], o.f[2], dz, wz);
                    const int off = 4 * (base + dx + __mul24(dy, px) + dz * pxy);
                    const float2 a0 = load_pair(gvol, off, 0);
                    const float2 a1 = load_pair(gvol, off, 4 * px);
                    const float2 c0v = load_pair(gvol, off, 4 * pxy);
                    const float2 c1v = load_pair(gvol, off, 4 * (pxy + px));
                    const float c00 = a0.x + wx * (a0.y - a0.x);
                    const float c10 = a1.x + wx * (a1.y - a1.x);
                    const float c01 = c0v.x + wx * (c0v.y - c0v.x);
                    const float c11 = c1v.x + wx * (c1v.y - c1v.x);
                    const float c0 = c00 + wy * (c10 - c00);
                    const float c1 = c01 + wy * (c11 - c01);
                    seg += c0 + wz * (c1 - c0);
                }
            }
            acc += (double)seg;
        }
    }
    double sq = 0.0;
    if (valid) {
        const long long idx = ((long long)k * nv + j) * nu + i;
        float val = (float)(acc * (double)step);
        if (Y) val -= Y[idx];
        out[idx] = val;
        sq = (double)val * (double)val;
    }
    if (partials) block_sum_store(sq, partials, tile);
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
    float Df[3];
    ray_setup(vc, dc, valid ? i : 0, valid ? j : 0, Q, D);
    to_float3(D, Df);
    int n0 = 1, n1 = 0;
    if (valid) ray_interval<T>(Q, D, Df, gc, n0, n1);
    const int px = gc.nx + 2;
    const int pxy = px * (gc.ny + 2);
    const double acc = march_double(Q, D, n0, n1, fp, px, pxy);
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

size_t tile_count(const cbct_geom &g) {
    return (size_t)((g.nu + TILE_U - 1) / TILE_U) * ((g.nv + TILE_V - 1) / TILE_V) * g.n_views;
}

// One-dimensional grid of all tiles of all views (see xcd_tile).
dim3 tile_grid(const cbct_plan &p) { return dim3((unsigned)tile_count(p.g)); }

// Cells of margin around the corner rays' box: the samples of rays inside a
// tile deviate from the corner rays' hull by at most t (1 - cos a) ~ t a^2/2,
// with a the tile's angular half-diagonal and t the largest sample distance
// inside the bordered grid: at most the source's distance to the grid
// centre (sad plus the grid's offset from the isocentre) plus half the
// grid's diagonal.
int tile_margin(const cbct_geom &g) {
    const double hd = sqrt(pow(0.5 * TILE_U * g.au, 2) + pow(0.5 * TILE_V * g.av, 2));
    const double a = hd / g.sdd;
    const double tmax = g.sad + sqrt(pow(g.x_off, 2) + pow(g.y_off, 2) + pow(g.z_off, 2)) +
                        sqrt(pow(0.5 * (g.nx + 2) * g.hx, 2) +
                             pow(0.5 * (g.ny + 2) * g.hy, 2) +
                             pow(0.5 * (g.nz + 2) * g.hz, 2));
    const double bulge = tmax * 0.5 * a * a * 1.01 / std::min(g.hx, std::min(g.hy, g.hz));
    return std::max(1, (int)ceil(bulge + 1e-3));
}

}  // namespace

int projector_tile_margin(const cbct_geom &g) { return tile_margin(g); }

void projector_config(int32_t out[4]) {
    out[0] = TILE_U;
    out[1] = TILE_V;
    out[2] = TILE_SUB;
    out[3] = TILE_LDS;
}

// Partial sums written by a float projection (one per workgroup of the
// tile grid); the double projector takes no partials.
size_t project_partials_count(const cbct_plan &p) { return tile_count(p.g); }
size_t project_partials_count(const cbct_geom &g) { return tile_count(g); }

size_t padded_count(const cbct_plan &p) {
    return (size_t)(p.g.nx + 2) * (p.g.ny + 2) * (p.g.nz + 2);
}


template <typename T>
hipError_t launch_pad(const cbct_plan &p, const T *f, T *fpad, hipStream_t s) {
    dim3 grid((p.g.nx + 2 + 31) / 32, (p.g.ny + 2 + 31) / 32, p.g.nz + 2);
    hipLaunchKernelGGL(k_pad<T>, grid, dim3(256), 0, s, f, fpad, p.g.nx, p.g.ny, p.g.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const cbct_plan &p, const T *fpad, const T *Y, T *out,
                          double *partials, hipStream_t s) {
    const long long elems = (long long)padded_count(p);
    if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL(k_project_tile, tile_grid(p), dim3(256), 0, s, p.d_views, p.det,
                           p.grid, p.g.nu, p.g.nv, fpad, (int)elems, Y, out, partials,
                           (float)p.g.step, tile_margin(p.g));
    } else {
        if (partials) return hipErrorInvalidValue;  // no partial sums in double
        hipLaunchKernelGGL(k_project<T>, project_grid(p), dim3(PROJ_BX, PROJ_BY), 0, s,
                           p.d_views, p.det, p.grid, p.g.nu, p.g.nv, fpad, Y, out, partials,
                           (T)p.g.step);
    }
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
