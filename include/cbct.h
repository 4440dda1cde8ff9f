/*
 * cbct.h - C ABI of the MI355X cone-beam CT reconstruction library.
 *
 * The library minimises E[f] = E1[f] + mu*E2[f] subject to f >= 0 (Eq. (1)
 * of Jia et al., "GPU-based fast cone beam CT reconstruction from
 * undersampled and noisy projection data via total variation"), where E1 is
 * the TV semi-norm (voxel mean of |grad f|) and E2 the mean squared
 * residual of the cone-beam projections, by the forward-backward splitting
 * of Algorithm A1 with a cascadic coarse-to-fine multigrid schedule.
 *
 * Units: lengths in mm, attenuation f in 1/mm, projections Y dimensionless
 * (line integrals).
 *
 * Conventions shared by every call:
 *   - Rotation axis z through the isocentre.  View k at angle theta_k
 *     (angles[k], or 2*pi*k/n_views when angles is NULL): source at
 *     R(theta)(0, -sad, 0); detector centre at R(theta)(0, sdd - sad, 0);
 *     detector u axis R(theta)(1, 0, 0), v axis z.
 *   - Pixel (i, j) centre: u = (i - (nu-1)/2) au + u_off,
 *     v = (j - (nv-1)/2) av + v_off.
 *   - Voxel (i, j, k) centre: x = (i - (nx-1)/2) hx + x_off, likewise y, z.
 *   - Volumes are float32 [nz][ny][nx] (x fastest); projection stacks are
 *     float32 [n_views][nv][nu] (u fastest).
 *   - Array arguments are DEVICE pointers owned by the caller; the library
 *     never frees them.  Host pointers are marked as such.
 *   - `stream` is a hipStream_t passed as void* (NULL = legacy default
 *     stream).  Calls are asynchronous on that stream unless stated:
 *     they return once the work is enqueued; results are valid after the
 *     stream synchronises.  Scratch memory is taken stream-ordered from a
 *     library-owned pool and returned on the same stream.
 *   - Return value 0 = success, or a negative CBCT_E* code; no C++
 *     exception crosses the ABI.  cbct_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 *   - Plans are immutable after creation except for the cached lambda (a
 *     guarded cache); they may be shared by threads and streams.  Solver
 *     states belong to one caller at a time.
 */
#ifndef CBCT_H
#define CBCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBCT_OK 0
#define CBCT_EINVAL (-1)     /* bad size, spacing, pointer or parameter */
#define CBCT_ENOMEM (-2)     /* device or host allocation failed */
#define CBCT_EHIP (-3)       /* HIP runtime or kernel launch error */
#define CBCT_ENONFINITE (-4) /* non-finite energy (only when traced) */

/* Scan and grid description.  `angles` is a host array of n_views radians
 * or NULL; it is copied at plan creation.  step is the ray sample spacing
 * Delta in mm; step <= 0 selects half the smallest voxel spacing.
 * u_off, v_off shift the detector in its own plane (mm, along e_u and
 * e_v): pixel (i, j) is centred at u = (i - (nu-1)/2) au + u_off,
 * v = (j - (nv-1)/2) av + v_off (u_off != 0 for half-fan scans).
 * x_off, y_off, z_off place the centre of the voxel grid (mm): voxel
 * (i, j, k) is centred at x = (i - (nx-1)/2) hx + x_off, and so on.  All
 * shifts are zero by default; they must be finite. */
typedef struct cbct_geom {
    int32_t nx, ny, nz;
    double hx, hy, hz;
    int32_t nu, nv;
    double au, av;
    double sad, sdd;
    int32_t n_views;
    const double *angles;
    double step;
    double u_off, v_off;
    double x_off, y_off, z_off;
} cbct_geom;

typedef struct cbct_plan cbct_plan;
typedef struct cbct_fbs_state cbct_fbs_state;

/* Create a plan: validates g (sizes > 0, spacings > 0, sdd > sad > 0,
 * the source outside the grid; limits: grid dimensions <= 32000, at most
 * 65535 views, a padded float volume below 2 GiB, and sample indices
 * (sdd + half the grid diagonal) / step <= 8e6), uploads per-view
 * constants, and counts the ray samples S.  EINVAL / ENOMEM / EHIP on
 * failure; *out untouched. */
int cbct_plan_create(const cbct_geom *g, cbct_plan **out);
void cbct_plan_destroy(cbct_plan *p);

/* Number of ray samples S = sum over rays of |N(r)| taken by one
 * projection (the work unit of the GRay-samples/s figures); -1 if p is
 * NULL. */
int64_t cbct_plan_samples(const cbct_plan *p);

/* The resolved geometry of the plan (step filled in); EINVAL on NULL. */
int cbct_plan_geom(const cbct_plan *p, cbct_geom *out);

/* Forward projection P of Eq. (1): y = P f, written over y.
 * (P f)_r = step * sum_n ftilde(s + n*step*e_r): samples at distances
 * n*step from the source along each source-to-pixel ray, ftilde the
 * trilinear interpolant of the grid, zero outside it.
 * f: [nz][ny][nx]; y: [n_views][nv][nu]. */
int cbct_project(const cbct_plan *p, const float *f, float *y, void *stream);

/* Forward projection fused with the residual needed by Step 1 of
 * Algorithm A1 (the paper computes P f - Y for every (u, v, theta) before
 * the per-voxel gradient): r = P f - Y.  If sumsq is not NULL it is a
 * device double that receives sum_r r^2 (for E2 = sumsq / N_meas). */
int cbct_project_residual(const cbct_plan *p, const float *f, const float *Y,
                          float *r, double *sumsq, void *stream);

/* Transpose of cbct_project (the matrix form of the gradient of E2 in the
 * paper's discussion of Eq. (2)), evaluated in gather form without atomics:
 * f = P^T y, written over f.  Deterministic: identical inputs give
 * bit-identical outputs. */
int cbct_backproject(const cbct_plan *p, const float *y, float *f, void *stream);

/* Step 1 of Algorithm A1 from a residual: g = f - tau * P^T r. */
int cbct_backproject_update(const cbct_plan *p, const float *r, const float *f,
                            double tau, float *g, void *stream);

/* The paper's gather-form gradient, Eq. (2), as an operator on residuals
 * y ([n_views][nv][nu], u fastest), on the scale of the matrix transpose:
 *   f(x_v) = hx hy hz / (au av) * sum_theta L^3 / (L0 l^2) * y~(u*, v*),
 * with (u*, v*) the imager point of the ray from the source through the
 * voxel centre x_v, l the source-voxel distance, L the source-imager-point
 * distance, L0 = sdd, and y~ the bilinear interpolant of the pixel-centre
 * values, zero beyond the outermost centres.  One lane per voxel, the
 * views summed in order: no atomics, deterministic.  It approximates
 * cbct_backproject (first order in the pixel pitch) and is not its exact
 * transpose.  f is written over; device pointers; EINVAL on NULL. */
int cbct_backproject_eq2(const cbct_plan *p, const float *y, float *f, void *stream);

/* Line integrals from detector counts, the step before the method:
 * y[i] = ln(ref / max(counts[i], min_count)) for i < n, with ref = flat[i]
 * (an open-beam flat field, same layout as counts) or, when flat is NULL,
 * ref = i0 for every pixel.  Evaluated in double, rounded to float.  Device
 * pointers; y may alias counts.  EINVAL for NULL counts or y, n < 0,
 * min_count <= 0, or (flat NULL and i0 <= 0). */
int cbct_log_counts(const float *counts, const float *flat, double i0, double min_count,
                    float *y, int64_t n, void *stream);

/* Float64 versions of cbct_project / cbct_backproject (same algorithm in
 * double precision; for derivative checks). */
int cbct_project_f64(const cbct_plan *p, const double *f, double *y, void *stream);
int cbct_backproject_f64(const cbct_plan *p, const double *y, double *f, void *stream);

/* Steps 2 and 3 of Algorithm A1: n_inner steps of projected gradient
 * descent on E1_eps[z] + (beta/2) E3[z], E3 = (1/V)||z - g||^2,
 *   z <- max(0, z - step * (D^T(Dz/|Dz|_eps) + beta (z - g)))
 * (no clipping when nonneg == 0), with D forward differences of physical
 * spacing (zero at the last index) and |.|_eps = sqrt(|.|^2 + eps^2).
 * Only grid->nx, ny, nz, hx, hy, hz are read.  f holds z0 on entry and
 * the result on exit; g is not modified.  step <= 0 selects
 * 1 / (beta + 4 (hx^-2 + hy^-2 + hz^-2) / eps).  beta > 0, eps > 0,
 * n_inner >= 0. */
int cbct_tv_prox(const cbct_geom *grid, const float *g, float *f, double beta,
                 double eps, int32_t n_inner, double step, int32_t nonneg,
                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweeps as cbct_tv_prox, same arguments and results bit for bit, with its
 * ping-pong volume in a fixed library array of 2^24 floats (64 MiB) held on
 * every GPU the library runs on until the process ends.  Grids of more
 * than 2^24 voxels give EINVAL (use cbct_tv_prox).  No device memory is
 * allocated or freed; the first call on a device looks up the array's
 * device address (EHIP if that fails), so make one call on each device
 * before capturing.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams, or threads) race and must be serialised by the caller.  The
 * launches are not recorded by cbct_kernel_timing. */
int cbct_tv_prox_noalloc(const cbct_geom *grid, const float *g, float *f, double beta,
                         double eps, int32_t n_inner, double step, int32_t nonneg,
                         void *stream);

/* E1 of Eq. (1) on the grid: out_host[0] = mean_v |Df|_v, out_host[1] =
 * mean_v sqrt(|Df|_v^2 + eps^2).  Synchronises `stream`. */
int cbct_tv_energy(const cbct_geom *grid, const float *f, double eps,
                   double *out_host, void *stream);

/* Largest eigenvalue of P^T P by power iteration from the all-ones vector
 * (n_iter steps, FP64 norms).  The result is cached in the plan per
 * n_iter.  Synchronises `stream`. */
int cbct_plan_lambda(const cbct_plan *p, int32_t n_iter, double *lambda_host,
                     void *stream);

/* Solver parameters.  E = E1 + mu*E2.  n_levels 1..CBCT_MAX_LEVELS
 * levels of the cascadic coarse-to-fine schedule (the paper's multigrid
 * remark): each coarser level has half the voxels per axis with doubled
 * spacing (2x2x2 block means of the finer start), a 2x2-binned detector
 * with doubled pitch and a doubled step.  Its cells and pixels sit at the
 * centres of the blocks they average: on an axis of odd size half a finer
 * spacing (pitch) below the finer grid's centre, the last finer plane
 * (row) belonging to no block.  Every level needs sizes >= 1.  Each
 * level's result is prolonged trilinearly into the next finer start.
 * iters[level] outer iterations, coarse first.  tol = 0 runs exactly
 * that many; tol > 0 ends a level after the first outer iteration with
 * ||f_{k+1} - f_k||_2 <= tol ||f_{k+1}||_2 (iters is then a maximum; one
 * host sync per outer iteration to read the change).  beta[level] <= 0
 * selects 1.1 * mu * (2 N_vox/N_meas) * lambda with lambda from 30
 * power-iteration steps on that level.  n_inner[level] <= 0 selects
 * min(200, ceil(3 (1 + 4 sum_a h_a^-2 / (eps beta)))).  eps is the TV
 * smoothing (1/mm^2).  trace_energy = 1 computes E at the start of every
 * outer iteration and at the end of each level (one host sync each);
 * trace_energy = 2 computes only the returned volume's E, at the end (one
 * projection and one host sync); 0 computes none; other values are
 * EINVAL.  gradient selects
 * Step 1's gradient of E2: 0 the exact transpose of the projector
 * (cbct_backproject; then E_eps never increases), 1 the paper's Eq. (2)
 * as printed (cbct_backproject_eq2, far cheaper, not matched). */
#define CBCT_MAX_LEVELS 4
typedef struct cbct_fbs_params {
    double mu;
    int32_t n_levels;
    int32_t iters[CBCT_MAX_LEVELS];
    double beta[CBCT_MAX_LEVELS];
    double eps;
    int32_t n_inner[CBCT_MAX_LEVELS];
    int32_t trace_energy;
    int32_t gradient;
    double tol;
} cbct_fbs_params;

/* Filled by the solver.  E, E_eps, E1, E2 describe the returned volume
 * (computed only when trace_energy is 1 or 2, else zero).  level_iters[level]
 * counts the outer iterations made on each level, iters_done their sum;
 * change[level] is the relative change of the level's last iteration
 * (tol > 0 only, else 0).  trace, if not NULL, is a caller HOST array of
 * at least sum over levels of (iters[level] + 1) rows of 4 doubles
 * (E, E_eps, E1, E2), filled when trace_energy = 1 and packed: level by
 * level, coarse first, (level_iters[level] + 1) rows each. */
typedef struct cbct_fbs_report {
    double E, E_eps, E1, E2;
    double beta_used[CBCT_MAX_LEVELS];
    int32_t n_inner_used[CBCT_MAX_LEVELS];
    int32_t level_iters[CBCT_MAX_LEVELS];
    int32_t iters_done;
    double change[CBCT_MAX_LEVELS];
    double *trace;
} cbct_fbs_report;

/* Full solve: f holds f0 on entry (each coarser level starts from the
 * 2x2x2 means of the next finer start) and the result on exit; Y is the
 * fine-level data.  Equivalent to init + step(all) + free.  Synchronises
 * `stream` before returning only when tracing, stopping by tolerance or
 * estimating beta. */
int cbct_fbs_solve(const cbct_plan *fine, const float *Y, float *f,
                   const cbct_fbs_params *prm, cbct_fbs_report *rep,
                   void *stream);

/* Step API for schedulers.  init validates, allocates the state (device
 * scratch for every level), bins Y and restricts f down the levels.
 * Y and f must stay valid until cbct_fbs_free.  step advances up to
 * n_iters outer iterations, moving to the next finer level (prolongation)
 * when a level is done; it is asynchronous unless tracing or stopping by
 * tolerance.  finished
 * returns 1 when every iteration is done, 0 otherwise, and a negative code
 * for a NULL state.  report copies the report so far. */
int cbct_fbs_init(const cbct_plan *fine, const float *Y, float *f,
                  const cbct_fbs_params *prm, cbct_fbs_state **out, void *stream);
int cbct_fbs_step(cbct_fbs_state *s, int32_t n_iters, void *stream);
int cbct_fbs_finished(const cbct_fbs_state *s);
int cbct_fbs_report_get(const cbct_fbs_state *s, cbct_fbs_report *rep);
void cbct_fbs_free(cbct_fbs_state *s);

/* Device bytes a solve of this geometry and schedule needs, including the
 * caller's Y and f arrays: the admission figure for schedulers.  When some
 * level's beta is to be estimated it includes the power iteration's scratch
 * for the finest level (held during init; an upper bound when the plan has
 * the estimate cached). */
size_t cbct_fbs_footprint(const cbct_geom *g, const cbct_fbs_params *prm);

/* Diagnostics: per-kernel device time.  cbct_kernel_timing(1) discards
 * earlier records and starts bracketing every library kernel launch with
 * two HIP events recorded on the launch stream; cbct_kernel_timing(0)
 * stops recording (records are kept).  cbct_kernel_timing_read waits for
 * the recorded events of one kernel kind and returns the number of
 * launches and their summed device time in ms (host pointers).  Process
 * wide; adds two event records per launch while enabled. */
#define CBCT_KERNEL_PAD 0        /* zero-bordered copy of the volume */
#define CBCT_KERNEL_PROJECT 1    /* ray march (P, optionally P f - Y) */
#define CBCT_KERNEL_CELLS 2      /* P^T pass 1: per-cell corner sums */
#define CBCT_KERNEL_GATHER 3     /* P^T pass 2: per-voxel sum (+ Step 1) */
#define CBCT_KERNEL_TV_SWEEP 4   /* one projected TV gradient step */
#define CBCT_KERNEL_TV_ENERGY 5  /* E1 partial sums */
#define CBCT_KERNEL_OTHER 6      /* reductions, fills, transfers */
#define CBCT_KERNEL_EQ2 7        /* Eq. (2) gradient (+ Step 1) */
#define CBCT_KERNEL_COUNT 8
int cbct_kernel_timing(int32_t enable);
int cbct_kernel_timing_read(int32_t kernel, int64_t *launches, double *total_ms);
/* The same for the kernel kinds whose bit (1 << kind) is set in mask: a
 * nonzero mask discards earlier records and records only those kinds (so
 * that the others run without events); 0 stops recording.  CBCT_EINVAL for
 * bits beyond CBCT_KERNEL_COUNT.  cbct_kernel_timing(e) is
 * cbct_kernel_timing_select(e ? all kinds : 0). */
int cbct_kernel_timing_select(uint32_t mask);

/* Diagnostics: sustained fused multiply-add rate of this device, the
 * measured ceiling of the ALU-bound kernels.  Runs one kernel of
 * independent non-packed FMA chains (no memory traffic in its loop) on
 * `stream`, in float32 (fp64 = 0) or float64 (fp64 = 1), times it with HIP
 * events and writes TFLOP/s (2 flop per FMA) to *tflops_host.  Allocates
 * and frees a small output buffer; synchronises `stream`. */
int cbct_probe_fma_rate(int32_t fp64, double *tflops_host, void *stream);

/* Diagnostics: the tunable sizes of the float kernels, written to the host
 * array out_host (at most n entries): [0] projector tile width and [1]
 * height in pixels, [2] samples per box (the projector stages runs of
 * such pieces), [3] LDS box capacity in floats; [4..6] transpose brick in
 * cells (x, y, z), [7] LDS table capacity in pixels.  A piece whose box
 * exceeds [3], or a brick whose footprint on the detector exceeds [7]
 * pixels, reads global memory instead of LDS (same results).  Returns the number of entries written (8 when n >= 8),
 * EINVAL for a NULL array or negative n.  No GPU work. */
int cbct_kernel_config(int32_t *out_host, int32_t n);

/* Diagnostics: the margin, in cells, by which the projector widens the box
 * its tile's four corner rays span over a chunk of samples, so that the
 * box holds every sample of the tile's other rays (they bulge out of the
 * corner rays' hull by at most t a^2 / 2 for a sample at distance t from the
 * source and a tile of angular half-diagonal a).  Written to *out_host for
 * geometry g; EINVAL for an invalid geometry or NULL pointer.  No GPU
 * work. */
int cbct_projector_tile_margin(const cbct_geom *g, int32_t *out_host);

const char *cbct_strerror(int code);
const char *cbct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_H */
