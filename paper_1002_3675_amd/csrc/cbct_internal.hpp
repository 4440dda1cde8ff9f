// Internal declarations of the MI355X cone-beam library: per-view constants,
// the ray/sample arithmetic shared by the projector and its transpose, and
// the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/cbct.h"

namespace cbct {

// Per-view constants, in voxel-index units where noted.  A sample n on the
// ray through pixel (u, v) lies at voxel-index coordinate
//     q_a(n) = Q_a + n * D_a,      D_a = (W_a + u U_a + v V_a) / |dir|,
// with |dir| = sqrt(sdd^2 + u^2 + v^2): the source-to-pixel direction
// sdd*e_w + u*e_u + v*e_v has orthonormal components.  Q is the source
// position in index coordinates, (s_a - x_a(0)) / h_a, and W, U, V are
// step/h_a times sdd*e_w, e_u and e_v.
struct ViewConst {
    float Q[3];
    float W[2];    // W_z = 0 (e_w lies in the xy plane)
    float U[2];    // U_z = 0
    float Vz;      // V_x = V_y = 0
    float src[2];  // source (mm), x and y; z = 0
    float cs, sn;  // cos(theta), sin(theta)
    double Qd[3];  // the same constants in double for the FP64 kernels
    double Wd[2], Ud[2], Vzd;
    double csd, snd;  // cos(theta), sin(theta) in double
};

// The dispatcher hands the workgroups of a launch to the 8 XCDs of the chip
// in turn by linear id, and each XCD has its own L2.  xcd_tile(b, n) maps
// linear workgroup id b of n to a tile id so that every XCD receives one
// contiguous range of tiles: neighbouring tiles, which read overlapping data,
// then share an L2.  It is a bijection of [0, n) whatever the dispatch order.
constexpr int XCDS = 8;

__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n / XCDS, r = n % XCDS;
    const int x = b % XCDS, i = b / XCDS;
    return x * q + (x < r ? x : r) + i;
}

struct DetConst {
    float u0, au, v0, av;  // pixel centre u = u0 + i*au, v = v0 + j*av (mm)
    float sdd2;            // sdd^2
    float sdd;
    double u0d, aud, v0d, avd, sdd2d, sddd;
};

struct GridConst {
    int nx, ny, nz;
    float hx, hy, hz;
    float x0, y0, z0;      // centre of voxel 0 (mm)
};

}  // namespace cbct

struct cbct_plan {
    cbct_geom g;                      // resolved (step filled, angles -> copy)
    std::vector<double> angles;
    cbct::ViewConst *d_views = nullptr;   // device [n_views]
    std::vector<cbct::ViewConst> h_views;
    cbct::DetConst det;
    cbct::GridConst grid;
    int64_t samples = 0;
    int device = 0;
    mutable std::mutex lam_mu;
    mutable std::vector<std::pair<int, double>> lam_cache;
    // next coarser multigrid level, created on first use
    mutable std::mutex coarse_mu;
    mutable cbct_plan *coarse = nullptr;
    // the transpose's geometry tables for the stand-alone operators,
    // prepared on first use (on that call's stream; bp_ready marks their
    // completion for other streams) and freed with the plan
    mutable std::mutex bp_mu;
    mutable void *bp_geom = nullptr;
    mutable hipEvent_t bp_ready = nullptr;
};

namespace cbct {

// ----------------------------------------------------------- errors --------
int set_error(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);

// ----------------------------------------------------------- memory --------
// Stream-ordered scratch from a library-owned pool on the current device.
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s);
hipError_t scratch_free(void *p, hipStream_t s);

// ----------------------------------------------------------- launchers -----
// All launchers enqueue on `s` and return the launch status.
template <typename T>
hipError_t launch_pad(const cbct_plan &p, const T *f, T *fpad, hipStream_t s);
template <typename T>
hipError_t launch_project(const cbct_plan &p, const T *fpad, const T *Y, T *out,
                          double *partials, hipStream_t s);
// The transpose needs the cell corner sums (bp_cells_bytes, written by
// launch_backproject_cells, read by launch_gather_cells) and the geometry
// tables (bp_geom_bytes: a per-pixel ray table and per-brick pixel
// rectangles), which depend on the plan only and are filled by
// launch_bp_prepare.  A combined workspace of bp_workspace_bytes holds the
// corner sums at offset 0 and the geometry tables at bp_geom_in.
size_t bp_cells_bytes(const cbct_geom &g, size_t elem_size);
size_t bp_geom_bytes(const cbct_geom &g);
size_t bp_workspace_bytes(const cbct_geom &g, size_t elem_size);
void *bp_geom_in(void *ws, const cbct_geom &g, size_t elem_size);
hipError_t launch_bp_prepare(const cbct_plan &p, void *geom, hipStream_t s);
template <typename T>
hipError_t launch_backproject_cells(const cbct_plan &p, const T *r, void *cells,
                                    const void *geom, hipStream_t s);
template <typename T>
hipError_t launch_gather_cells(const cbct_plan &p, const void *ws, const T *f, double tau,
                               T *out, hipStream_t s);
// Eq. (2) gradient of the residual r: out = B r, or out = f - tau * B r
// when f is given
hipError_t launch_eq2(const cbct_plan &p, const float *r, const float *f, double tau,
                      float *out, hipStream_t s);
hipError_t launch_count_samples(const cbct_plan &p, unsigned long long *count, hipStream_t s);

// Tunable sizes of the float kernels (diagnostics): the projector's tile
// width and height in pixels, samples per chunk and LDS box in floats; the
// transpose's brick in cells (x, y, z) and LDS table in pixels.
void projector_config(int32_t out[4]);
int projector_tile_margin(const cbct_geom &g);
void cell_pass_config(int32_t out[4]);

size_t project_partials_count(const cbct_plan &p);
size_t project_partials_count(const cbct_geom &g);
size_t padded_count(const cbct_plan &p);

hipError_t launch_tv_sweep(const GridConst &gc, const float *z, const float *g, float *out,
                           float beta, float eps, float step, int nonneg, hipStream_t s);
hipError_t launch_tv_energy(const GridConst &gc, const float *z, double eps,
                            double *partials, int *n_partials, hipStream_t s);
hipError_t launch_reduce_sum(const double *partials, int n, double *out, int n_out_cols,
                             hipStream_t s);
size_t tv_energy_partials_count(const GridConst &gc);

// Per-block partial sums (sum (a - b)^2, sum a^2), two doubles per block,
// at most DIFF_BLOCKS blocks: the relative change of an outer iteration.
constexpr int DIFF_BLOCKS = 1024;
hipError_t launch_diff_sums(const float *a, const float *b, size_t n, double *partials,
                            int *n_partials, hipStream_t s);
hipError_t launch_sumsq(const float *x, size_t n, double *partials, int *n_partials,
                        hipStream_t s);
hipError_t launch_fill(float *x, size_t n, float v, hipStream_t s);
hipError_t launch_log_counts(const float *counts, const float *flat, double i0,
                             double min_count, float *y, long long n, hipStream_t s);
// FMA-rate probe: blocks x 256 lanes, iters x 8 FMAs each, into out
// (blocks x 256 elements of float, or of double when fp64)
hipError_t launch_probe_fma(bool fp64, void *out, int blocks, int iters, hipStream_t s);
hipError_t launch_scale(const float *x, size_t n, const double *denom, float *out,
                        hipStream_t s);
hipError_t launch_bin_detector(const float *y, int nu, int nv, int nviews, float *out,
                               hipStream_t s);
hipError_t launch_restrict(const float *f, int nx, int ny, int nz, float *out, hipStream_t s);
hipError_t launch_prolong(const float *fc, int cx, int cy, int cz, float *ff, int nx, int ny,
                          int nz, hipStream_t s);

GridConst grid_of(const cbct_geom &g);

}  // namespace cbct
