/*
 * FP64 reference ("oracle") for TV-regularised cone-beam CT reconstruction
 * by forward-backward splitting (Jia, Lou, Li, Song, Jiang, "GPU-based fast
 * cone beam CT reconstruction from undersampled and noisy projection data
 * via total variation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow, obviously correct
 * C99 + OpenMP in double precision.  It shares no code with the HIP library
 * and is used only by the test-suite, the smoke check and the CPU baseline
 * of the benchmark.  No product code path may call it.
 *
 * Every function follows one passage of the paper:
 *   Eq. (1)                    E = E1 + mu*E2 subject to f >= 0
 *   E1, E2 definitions         E1 = (1/V)||grad f||_1,
 *                              E2 = (1/(N_theta*A)) sum_theta ||P f - Y||^2
 *   Algorithm A1               update / minimise / correct
 *   Eq. (2) and text around it the gradient of E2 needs P and its transpose
 *   multi-grid remark          coarse-to-fine schedule
 * The discretisation choices the paper leaves open are fixed as follows
 * (each is a reading, not something the paper states):
 *   P      uniform sample spacing `step` along each source ray, samples at
 *          distance n*step from the source (n integer), trilinear
 *          interpolation of the voxel grid with zero outside it;
 *          (P f)_r = step * sum_n ftilde(s + n*step*e_r).
 *   P^T    the matrix transpose of that P, applied by scattering.
 *   grad   forward differences with physical spacing, zero at the last
 *          index of each axis; E1 is the voxel mean of the isotropic
 *          |grad f| (optionally smoothed: sqrt(|grad f|^2 + eps^2)).
 *   E2     mean of squared residuals over all detector pixels and views.
 *   Step 1 g = f - tau * P^T (P f - Y), tau = (mu/beta) * 2 N_vox / N_meas
 *          (the functional derivative is 1/(voxel volume) times the partial
 *          derivative, and V / voxel volume = N_vox).
 *   Step 2 projected gradient descent on E1_eps + (beta/2) E3 started from
 *          the current f; Step 3 (clip at zero) is applied inside each inner
 *          step (clip_mode 0) or once after the inner loop (clip_mode 1,
 *          the literal order of Algorithm A1).
 *   beta   1.1 * mu * (2 N_vox/N_meas) * lambda, lambda from power
 *          iteration on P^T P started from the all-ones vector, unless the
 *          caller gives beta.
 *   multi-grid  up to four levels, cascadic: each coarser level has half
 *          the voxels per axis (spacing doubled, 2x2x2 block means), a
 *          2x2-binned detector (pitch doubled) and the step doubled; its
 *          cells and pixels sit at the centres of the blocks and pixel
 *          pairs they average (a half fine pitch off the axis when a size
 *          is odd, the last fine plane then left out); each level's result
 *          is prolonged trilinearly (cell-centred) to the next finer grid.
 *   stopping  fixed outer counts per level, or, with tol > 0, a level
 *          stops after the first iteration with
 *          ||f_{k+1} - f_k||_2 <= tol * ||f_{k+1}||_2 (the count is then a
 *          maximum).
 *
 * Parameter packing used by every entry point:
 *   dims[6] = {nx, ny, nz, nu, nv, n_views}
 *   par[13] = {hx, hy, hz, au, av, sad, sdd, step, u_off, v_off,
 *              x_off, y_off, z_off}
 *             (step <= 0: half the smallest voxel spacing; u_off, v_off
 *             shift the detector in its plane, x_off, y_off, z_off the
 *             volume centre, in mm)
 *   angles  = n_views radians, or NULL for 2*pi*k/n_views.
 * Volumes are [nz][ny][nx] (x fastest); projections [n_views][nv][nu].
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz, nu, nv, nviews;
    double hx, hy, hz, au, av, sad, sdd, step;
    double u_off, v_off;  /* detector shift in its plane (mm) */
    double off[3];        /* volume centre (mm) */
    const double *angles;
} geom_t;

static geom_t unpack(const int *dims, const double *par, const double *angles)
{
    geom_t g;
    g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
    g.nu = dims[3]; g.nv = dims[4]; g.nviews = dims[5];
    g.hx = par[0]; g.hy = par[1]; g.hz = par[2];
    g.au = par[3]; g.av = par[4]; g.sad = par[5]; g.sdd = par[6];
    g.step = par[7];
    g.u_off = par[8];
    g.v_off = par[9];
    g.off[0] = par[10];
    g.off[1] = par[11];
    g.off[2] = par[12];
    if (g.step <= 0.0) {
        double m = g.hx;
        if (g.hy < m) m = g.hy;
        if (g.hz < m) m = g.hz;
        g.step = 0.5 * m;
    }
    g.angles = angles;
    return g;
}

static double view_angle(const geom_t *g, int k)
{
    if (g->angles) return g->angles[k];
    return 2.0 * M_PI * (double)k / (double)g->nviews;
}

/* Source position and unit direction of the ray through pixel (i, j) of
 * view k (geometry of the paper's Eq. (2): the ray from the source to the
 * imager point (u, v); the imager sits SDD from the source). */
static void ray_of(const geom_t *g, int k, int i, int j, double s[3], double e[3])
{
    double th = view_angle(g, k), c = cos(th), sn = sin(th);
    double u = ((double)i - 0.5 * (g->nu - 1)) * g->au + g->u_off;
    double v = ((double)j - 0.5 * (g->nv - 1)) * g->av + g->v_off;
    double d[3];
    s[0] = g->sad * sn;  s[1] = -g->sad * c;  s[2] = 0.0;
    /* detector point = centre R(th)(0, SDD-SAD, 0) + u*R(th)(1,0,0) + v*z */
    d[0] = -(g->sdd - g->sad) * sn + u * c;
    d[1] = (g->sdd - g->sad) * c + u * sn;
    d[2] = v;
    double L = sqrt((d[0] - s[0]) * (d[0] - s[0]) + (d[1] - s[1]) * (d[1] - s[1])
                    + (d[2] - s[2]) * (d[2] - s[2]));
    for (int a = 0; a < 3; ++a) e[a] = (d[a] - s[a]) / L;
}

/* Range of sample indices n with n*step inside the ray's intersection with
 * the box on which the zero-padded trilinear interpolant can be non-zero,
 * |x_a - off_a| <= (N_a + 1) h_a / 2.  Returns 0 when the ray misses it. */
static int sample_range(const geom_t *g, const double s[3], const double e[3],
                        long *n0, long *n1)
{
    double half[3] = {0.5 * (g->nx + 1) * g->hx, 0.5 * (g->ny + 1) * g->hy,
                      0.5 * (g->nz + 1) * g->hz};
    double tin = -INFINITY, tout = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (e[a] == 0.0) {
            if (s[a] <= g->off[a] - half[a] || s[a] >= g->off[a] + half[a]) return 0;
            continue;
        }
        double t1 = (g->off[a] - half[a] - s[a]) / e[a];
        double t2 = (g->off[a] + half[a] - s[a]) / e[a];
        double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
        if (lo > tin) tin = lo;
        if (hi < tout) tout = hi;
    }
    if (!(tin <= tout)) return 0;
    *n0 = (long)ceil(tin / g->step);
    *n1 = (long)floor(tout / g->step);
    return *n0 <= *n1;
}

/* Trilinear interpolation stencil at point p: base index (i0,j0,k0) and the
 * per-axis weights of the two neighbours along each axis. */
static void stencil(const geom_t *g, const double p[3], long idx0[3], double w[3][2])
{
    double h[3] = {g->hx, g->hy, g->hz};
    int n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a) {
        double q = (p[a] - g->off[a]) / h[a] + 0.5 * (n[a] - 1);  /* voxel-index coordinate */
        double fl = floor(q);
        idx0[a] = (long)fl;
        w[a][1] = q - fl;
        w[a][0] = 1.0 - w[a][1];
    }
}

/* ------------------------------------------------------- Eq. (2) ---- */

/* The paper's gather-form gradient, Eq. (2), as an operator on residuals
 * y ([n_views][nv][nu]) with the scale of the matrix transpose:
 *   out(x_v) = (hx hy hz / (au av)) * sum_theta L^3 / (L0 l^2) * y~(u*, v*)
 * where, for view theta, (u*, v*) is the imager point on the ray from the
 * source through the voxel centre x_v, l = |x_v - s| the source-voxel
 * distance, L = sqrt(L0^2 + u*^2 + v*^2) the source-imager-point distance
 * and L0 = SDD.  (hx hy hz / (au av)) * (P^theta)^* approximates the
 * discrete transpose (the sum over pixels is (1/(au av)) times the
 * imager integral, the sum over voxels (1/(hx hy hz)) times the volume
 * integral), so Step 1 keeps the form g = f - tau * out.
 * y~ is the bilinear interpolant of the pixel-centre values, zero beyond
 * the outermost pixel centres (the paper leaves the interpolation open). */
void or_eq2_backproject(const int *dims, const double *par, const double *angles,
                        const double *y, double *out)
{
    geom_t g = unpack(dims, par, angles);
    double scale = g.hx * g.hy * g.hz / (g.au * g.av);
    long nvox = (long)g.nx * g.ny * g.nz;
#pragma omp parallel for schedule(static)
    for (long v = 0; v < nvox; ++v) {
        long i = v % g.nx, j = (v / g.nx) % g.ny, k = v / ((long)g.nx * g.ny);
        double x = ((double)i - 0.5 * (g.nx - 1)) * g.hx + g.off[0];
        double yy = ((double)j - 0.5 * (g.ny - 1)) * g.hy + g.off[1];
        double z = ((double)k - 0.5 * (g.nz - 1)) * g.hz + g.off[2];
        double sum = 0.0;
        for (int t = 0; t < g.nviews; ++t) {
            double th = view_angle(&g, t), c = cos(th), sn = sin(th);
            /* source (sad sin, -sad cos, 0); imager axes e_u = (cos, sin, 0),
             * e_v = z; the central ray runs along e_w = (-sin, cos, 0) */
            double wx = x - g.sad * sn, wy = yy + g.sad * c, wz = z;
            double depth = -wx * sn + wy * c;
            double us = g.sdd * (wx * c + wy * sn) / depth;
            double vs = g.sdd * wz / depth;
            double l2 = wx * wx + wy * wy + wz * wz;
            double L = sqrt(g.sdd * g.sdd + us * us + vs * vs);
            double w = L * L * L / (g.sdd * l2);
            double fi = (us - g.u_off) / g.au + 0.5 * (g.nu - 1);
            double fj = (vs - g.v_off) / g.av + 0.5 * (g.nv - 1);
            double i0 = floor(fi), j0 = floor(fj), a = fi - i0, b = fj - j0;
            const double *yt = y + (long)t * g.nu * g.nv;
            double val = 0.0;
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    long ii = (long)i0 + di, jj = (long)j0 + dj;
                    if (ii < 0 || ii >= g.nu || jj < 0 || jj >= g.nv) continue;
                    val += (di ? a : 1.0 - a) * (dj ? b : 1.0 - b) * yt[jj * g.nu + ii];
                }
            sum += w * val;
        }
        out[v] = scale * sum;
    }
}

/* ---------------------------------------------------------------- P ---- */

/* y = P f: the discrete cone-beam projection P^theta of Eq. (1), for every
 * view theta and imager pixel (u, v). */
void or_project(const int *dims, const double *par, const double *angles,
                const double *f, double *y)
{
    geom_t g = unpack(dims, par, angles);
    long nrays = (long)g.nviews * g.nv * g.nu;
#pragma omp parallel for schedule(dynamic, 64)
    for (long r = 0; r < nrays; ++r) {
        int i = (int)(r % g.nu), j = (int)((r / g.nu) % g.nv), k = (int)(r / ((long)g.nu * g.nv));
        double s[3], e[3];
        ray_of(&g, k, i, j, s, e);
        long n0, n1;
        double sum = 0.0;
        if (sample_range(&g, s, e, &n0, &n1)) {
            for (long n = n0; n <= n1; ++n) {
                double t = (double)n * g.step, p[3];
                for (int a = 0; a < 3; ++a) p[a] = s[a] + t * e[a];
                long b[3]; double w[3][2];
                stencil(&g, p, b, w);
                for (int dz = 0; dz < 2; ++dz) {
                    long kz = b[2] + dz;
                    if (kz < 0 || kz >= g.nz) continue;
                    for (int dy = 0; dy < 2; ++dy) {
                        long jy = b[1] + dy;
                        if (jy < 0 || jy >= g.ny) continue;
                        for (int dx = 0; dx < 2; ++dx) {
                            long ix = b[0] + dx;
                            if (ix < 0 || ix >= g.nx) continue;
                            sum += w[0][dx] * w[1][dy] * w[2][dz]
                                   * f[ix + g.nx * (jy + g.ny * kz)];
                        }
                    }
                }
            }
        }
        y[r] = g.step * sum;
    }
}

/* Exact number of samples S = sum_r |N(r)| taken by P (the work unit of
 * the throughput figures). */
long long or_count_samples(const int *dims, const double *par, const double *angles)
{
    geom_t g = unpack(dims, par, angles);
    long nrays = (long)g.nviews * g.nv * g.nu;
    long long total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (long r = 0; r < nrays; ++r) {
        int i = (int)(r % g.nu), j = (int)((r / g.nu) % g.nv), k = (int)(r / ((long)g.nu * g.nv));
        double s[3], e[3];
        ray_of(&g, k, i, j, s, e);
        long n0, n1;
        if (sample_range(&g, s, e, &n0, &n1)) total += n1 - n0 + 1;
    }
    return total;
}

/* -------------------------------------------------------------- P^T ---- */

/* f = P^T y, the transpose of or_project written as the plain scatter that
 * the paper describes as the straightforward matrix form of the gradient of
 * E2 (the form with write conflicts on a GPU).  Each thread scatters into
 * a private volume; the private volumes are summed in thread order. */
void or_backproject(const int *dims, const double *par, const double *angles,
                    const double *y, double *f)
{
    geom_t g = unpack(dims, par, angles);
    long nvox = (long)g.nx * g.ny * g.nz;
    long nrays = (long)g.nviews * g.nv * g.nu;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * (size_t)nvox, sizeof(double));
    if (!priv) { memset(f, 0xff, sizeof(double) * (size_t)nvox); return; }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = priv + (size_t)tid * (size_t)nvox;
#pragma omp for schedule(static)
        for (long r = 0; r < nrays; ++r) {
            if (y[r] == 0.0) continue;
            int i = (int)(r % g.nu), j = (int)((r / g.nu) % g.nv), k = (int)(r / ((long)g.nu * g.nv));
            double s[3], e[3];
            ray_of(&g, k, i, j, s, e);
            long n0, n1;
            if (!sample_range(&g, s, e, &n0, &n1)) continue;
            double yr = g.step * y[r];
            for (long n = n0; n <= n1; ++n) {
                double t = (double)n * g.step, p[3];
                for (int a = 0; a < 3; ++a) p[a] = s[a] + t * e[a];
                long b[3]; double w[3][2];
                stencil(&g, p, b, w);
                for (int dz = 0; dz < 2; ++dz) {
                    long kz = b[2] + dz;
                    if (kz < 0 || kz >= g.nz) continue;
                    for (int dy = 0; dy < 2; ++dy) {
                        long jy = b[1] + dy;
                        if (jy < 0 || jy >= g.ny) continue;
                        for (int dx = 0; dx < 2; ++dx) {
                            long ix = b[0] + dx;
                            if (ix < 0 || ix >= g.nx) continue;
                            acc[ix + g.nx * (jy + g.ny * kz)] += yr * w[0][dx] * w[1][dy] * w[2][dz];
                        }
                    }
                }
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (long v = 0; v < nvox; ++v) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += priv[(size_t)t * (size_t)nvox + v];
        f[v] = s;
    }
    free(priv);
}

/* --------------------------------------------------- gradient and TV ---- */

/* D: forward differences (z[i+e_a] - z[i]) / h_a, zero at the last index. */
void or_grad(const int *vdims, const double *h, const double *z,
             double *gx, double *gy, double *gz)
{
    int nx = vdims[0], ny = vdims[1], nz = vdims[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                gx[v] = (i < nx - 1) ? (z[v + 1] - z[v]) / h[0] : 0.0;
                gy[v] = (j < ny - 1) ? (z[v + nx] - z[v]) / h[1] : 0.0;
                gz[v] = (k < nz - 1) ? (z[v + (long)nx * ny] - z[v]) / h[2] : 0.0;
            }
}

/* D^T: the exact adjoint of or_grad. */
void or_grad_adjoint(const int *vdims, const double *h, const double *px,
                     const double *py, const double *pz, double *out)
{
    int nx = vdims[0], ny = vdims[1], nz = vdims[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                double s = 0.0;
                if (i > 0) s += px[v - 1] / h[0];
                if (i < nx - 1) s -= px[v] / h[0];
                if (j > 0) s += py[v - nx] / h[1];
                if (j < ny - 1) s -= py[v] / h[1];
                if (k > 0) s += pz[v - (long)nx * ny] / h[2];
                if (k < nz - 1) s -= pz[v] / h[2];
                out[v] = s;
            }
}

/* E1 of Eq. (1) as a voxel mean: (1/N_vox) sum_v sqrt(|D z|_v^2 + eps^2);
 * eps = 0 gives the TV semi-norm itself. */
double or_tv(const int *vdims, const double *h, const double *z, double eps)
{
    int nx = vdims[0], ny = vdims[1], nz = vdims[2];
    long nvox = (long)nx * ny * nz;
    double total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (long k = 0; k < nz; ++k) {
        double slab = 0.0;
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                double a = (i < nx - 1) ? (z[v + 1] - z[v]) / h[0] : 0.0;
                double b = (j < ny - 1) ? (z[v + nx] - z[v]) / h[1] : 0.0;
                double c = (k < nz - 1) ? (z[v + (long)nx * ny] - z[v]) / h[2] : 0.0;
                slab += sqrt(a * a + b * b + c * c + eps * eps);
            }
        total += slab;
    }
    return total / (double)nvox;
}

/* D^T (D z / |D z|_eps): N_vox times the gradient of the smoothed E1. */
void or_tv_grad(const int *vdims, const double *h, const double *z, double eps,
                double *out)
{
    long nvox = (long)vdims[0] * vdims[1] * vdims[2];
    double *px = (double *)malloc(sizeof(double) * (size_t)nvox * 3);
    double *py = px + nvox, *pz = py + nvox;
    or_grad(vdims, h, z, px, py, pz);
#pragma omp parallel for schedule(static)
    for (long v = 0; v < nvox; ++v) {
        double m = sqrt(px[v] * px[v] + py[v] * py[v] + pz[v] * pz[v] + eps * eps);
        px[v] /= m; py[v] /= m; pz[v] /= m;
    }
    or_grad_adjoint(vdims, h, px, py, pz, out);
    free(px);
}

/* Step size 1 / Lipschitz of the inner objective: beta + ||D||^2/eps with
 * ||D||^2 <= 4 * sum_a h_a^-2. */
double or_prox_step(const double *h, double beta, double eps, double tv_weight)
{
    double d2 = 4.0 * (1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]));
    return 1.0 / (beta + tv_weight * d2 / eps);
}

/* Algorithm A1, Steps 2 and 3: minimise E1_eps[z] + (beta/2) E3[z],
 * E3 = (1/V)||z - g||^2, by gradient descent from the z given on input.
 *   clip_mode 0: z <- max(0, z - s*grad) every inner step (projected GD);
 *   clip_mode 1: plain GD for n_inner steps, then z <- max(0, z) once;
 *   clip_mode 2: plain GD, no clipping.
 * tv_weight scales E1 (1 in the method; 0 reduces Step 2 to z = g).
 * step <= 0 selects or_prox_step.  phi (optional, n_inner+1 entries)
 * receives E1_eps + (beta/2) E3 before each step and after the last. */
void or_tv_prox(const int *vdims, const double *h, const double *g, double *z,
                double beta, double eps, int n_inner, double step, int clip_mode,
                double tv_weight, double *phi)
{
    long nvox = (long)vdims[0] * vdims[1] * vdims[2];
    if (step <= 0.0) step = or_prox_step(h, beta, eps, tv_weight);
    double *tg = (double *)malloc(sizeof(double) * (size_t)nvox);
    for (int m = 0; m <= n_inner; ++m) {
        if (phi) {
            double e3 = 0.0;
            for (long v = 0; v < nvox; ++v) e3 += (z[v] - g[v]) * (z[v] - g[v]);
            phi[m] = tv_weight * or_tv(vdims, h, z, eps) + 0.5 * beta * e3 / (double)nvox;
        }
        if (m == n_inner) break;
        if (tv_weight != 0.0) or_tv_grad(vdims, h, z, eps, tg);
        else memset(tg, 0, sizeof(double) * (size_t)nvox);
#pragma omp parallel for schedule(static)
        for (long v = 0; v < nvox; ++v) {
            double zn = z[v] - step * (tv_weight * tg[v] + beta * (z[v] - g[v]));
            if (clip_mode == 0 && zn < 0.0) zn = 0.0;
            z[v] = zn;
        }
    }
    if (clip_mode == 1)
        for (long v = 0; v < nvox; ++v)
            if (z[v] < 0.0) z[v] = 0.0;
    free(tg);
}

/* ------------------------------------------------------ data term ------ */

/* E2 of Eq. (1): mean over views and pixels of (P f - Y)^2.  r receives
 * the residual P f - Y when not NULL. */
double or_data_energy(const int *dims, const double *par, const double *angles,
                      const double *f, const double *Y, double *r)
{
    geom_t g = unpack(dims, par, angles);
    long nmeas = (long)g.nviews * g.nu * g.nv;
    double *res = r ? r : (double *)malloc(sizeof(double) * (size_t)nmeas);
    or_project(dims, par, angles, f, res);
    double s = 0.0;
    for (long i = 0; i < nmeas; ++i) {
        res[i] -= Y[i];
        s += res[i] * res[i];
    }
    if (!r) free(res);
    return s / (double)nmeas;
}

/* Largest eigenvalue of P^T P by power iteration from the all-ones vector:
 * x <- P^T P x / ||P^T P x||; returns ||P^T P x|| of the last step. */
double or_power_lambda(const int *dims, const double *par, const double *angles,
                       int n_iter)
{
    geom_t g = unpack(dims, par, angles);
    long nvox = (long)g.nx * g.ny * g.nz, nmeas = (long)g.nviews * g.nu * g.nv;
    double *x = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *w = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *y = (double *)malloc(sizeof(double) * (size_t)nmeas);
    double inv = 1.0 / sqrt((double)nvox), lam = 0.0;
    for (long v = 0; v < nvox; ++v) x[v] = inv;
    for (int it = 0; it < n_iter; ++it) {
        or_project(dims, par, angles, x, y);
        or_backproject(dims, par, angles, y, w);
        double n2 = 0.0;
        for (long v = 0; v < nvox; ++v) n2 += w[v] * w[v];
        lam = sqrt(n2);
        for (long v = 0; v < nvox; ++v) x[v] = w[v] / lam;
    }
    free(x); free(w); free(y);
    return lam;
}

/* --------------------------------------------------- multi-grid -------- */

/* Coarse detector: mean of each 2x2 pixel block (nu, nv even). */
void or_bin_detector(int nu, int nv, int nviews, const double *y, double *yc)
{
    int cu = nu / 2, cv = nv / 2;
    for (long k = 0; k < nviews; ++k)
        for (long j = 0; j < cv; ++j)
            for (long i = 0; i < cu; ++i) {
                const double *b = y + (size_t)k * nu * nv + (size_t)(2 * j) * nu + 2 * i;
                yc[(size_t)k * cu * cv + (size_t)j * cu + i] = 0.25 * (b[0] + b[1] + b[nu] + b[nu + 1]);
            }
}

/* Coarse volume: mean of each 2x2x2 voxel block. */
void or_restrict(const int *fdims, const double *ff, double *fc)
{
    int nx = fdims[0], ny = fdims[1], nz = fdims[2];
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (long k = 0; k < cz; ++k)
        for (long j = 0; j < cy; ++j)
            for (long i = 0; i < cx; ++i) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += ff[(2 * i + a) + (long)nx * ((2 * j + b) + (long)ny * (2 * k + c))];
                fc[i + cx * (j + cy * k)] = 0.125 * s;
            }
}

/* Fine volume by trilinear interpolation of the coarse one at the fine
 * voxel centres: fine index i sits at coarse coordinate (i + 1/2)/2 - 1/2,
 * clamped to the coarse grid. */
void or_prolong(const int *cdims, const int *fdims, const double *fc, double *ff)
{
    int cn[3] = {cdims[0], cdims[1], cdims[2]};
    int fn[3] = {fdims[0], fdims[1], fdims[2]};
    for (long k = 0; k < fn[2]; ++k)
        for (long j = 0; j < fn[1]; ++j)
            for (long i = 0; i < fn[0]; ++i) {
                long fi[3] = {i, j, k};
                long b[3]; double w[3];
                for (int a = 0; a < 3; ++a) {
                    double c = (fi[a] + 0.5) / 2.0 - 0.5;
                    if (c < 0.0) c = 0.0;
                    if (c > cn[a] - 1) c = cn[a] - 1;
                    long c0 = (long)floor(c);
                    if (c0 > cn[a] - 2) c0 = cn[a] - 2;
                    if (c0 < 0) c0 = 0;
                    b[a] = c0;
                    w[a] = (cn[a] > 1) ? c - (double)c0 : 0.0;
                }
                double s = 0.0;
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            double wt = (dx ? w[0] : 1 - w[0]) * (dy ? w[1] : 1 - w[1]) * (dz ? w[2] : 1 - w[2]);
                            if (wt == 0.0) continue;
                            long ix = b[0] + dx, jy = b[1] + dy, kz = b[2] + dz;
                            s += wt * fc[ix + cn[0] * (jy + (long)cn[1] * kz)];
                        }
                ff[i + fn[0] * (j + (long)fn[1] * k)] = s;
            }
}

/* ------------------------------------------------------- solver -------- */

/* Inner iteration count when the caller gives none: enough steps that the
 * contraction (1 - step*beta)^K is below e^-3, at most 200. */
int or_default_inner(const double *h, double beta, double eps)
{
    double d2 = 4.0 * (1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]));
    double k = ceil(3.0 * (1.0 + d2 / (eps * beta)));
    return k > 200.0 ? 200 : (int)k;
}

/* Energies of f for trace/report: out[0..3] = E, E_eps, E1, E2. */
static void energies(const int *dims, const double *par, const double *angles,
                     const double *f, const double *Y, double mu, double eps, double *out)
{
    double h[3] = {par[0], par[1], par[2]};
    double e2 = or_data_energy(dims, par, angles, f, Y, NULL);
    double e1 = or_tv(dims, h, f, 0.0), e1e = or_tv(dims, h, f, eps);
    out[0] = e1 + mu * e2;
    out[1] = e1e + mu * e2;
    out[2] = e1;
    out[3] = e2;
}

/* Relative change ||a - b||_2 / ||a||_2 of one outer iteration (a the new
 * iterate, b the previous one); 0 when both are zero, +inf when only a
 * is. */
static double rel_change(long n, const double *a, const double *b)
{
    double d = 0.0, m = 0.0;
    for (long v = 0; v < n; ++v) {
        d += (a[v] - b[v]) * (a[v] - b[v]);
        m += a[v] * a[v];
    }
    if (m == 0.0) return d == 0.0 ? 0.0 : INFINITY;
    return sqrt(d / m);
}

/* One level of Algorithm A1: at most iters outer iterations on f (in
 * place); with tol > 0 it stops after the first iteration whose relative
 * change is <= tol.  Returns the number of iterations made; *change gets
 * the relative change of the last one (0 if none, or if tol <= 0). */
static int fbs_level(const int *dims, const double *par, const double *angles,
                     const double *Y, double *f, double mu, double beta, double eps,
                     int n_inner, int iters, double tol, double tv_weight, int clip_mode,
                     int grad_mode, double *trace, double *change)
{
    geom_t g = unpack(dims, par, angles);
    long nvox = (long)g.nx * g.ny * g.nz, nmeas = (long)g.nviews * g.nu * g.nv;
    double h[3] = {g.hx, g.hy, g.hz};
    double tau = (mu / beta) * 2.0 * (double)nvox / (double)nmeas;
    double *r = (double *)malloc(sizeof(double) * (size_t)nmeas);
    double *grad = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *gaux = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *prev = tol > 0.0 ? (double *)malloc(sizeof(double) * (size_t)nvox) : NULL;
    int it = 0;
    *change = 0.0;
    while (it < iters) {
        if (trace) energies(dims, par, angles, f, Y, mu, eps, trace + 4 * it);
        if (prev) memcpy(prev, f, sizeof(double) * (size_t)nvox);
        /* Step 1 (update): g = f - (mu V / beta) dE2/df */
        or_data_energy(dims, par, angles, f, Y, r);
        if (grad_mode == 1)
            or_eq2_backproject(dims, par, angles, r, grad);  /* Eq. (2) as printed */
        else
            or_backproject(dims, par, angles, r, grad);      /* matched transpose */
        for (long v = 0; v < nvox; ++v) gaux[v] = f[v] - tau * grad[v];
        /* Steps 2 and 3 (minimise, correct), started from the current f */
        or_tv_prox(dims, h, gaux, f, beta, eps, n_inner, 0.0, clip_mode, tv_weight, NULL);
        ++it;
        if (prev) {
            *change = rel_change(nvox, f, prev);
            if (*change <= tol) break;
        }
    }
    if (trace) energies(dims, par, angles, f, Y, mu, eps, trace + 4 * it);
    free(r); free(grad); free(gaux); free(prev);
    return it;
}

/* Geometry of the next coarser level: half the voxels per axis with the
 * spacing doubled, a detector of half the pixels per axis with the pitch
 * doubled, the step doubled.  A coarse cell is the mean of fine voxels
 * (2i, 2i + 1) along each axis, so it is placed at their centre: on an axis
 * of odd size that is half a fine spacing below the fine grid's centre
 * (the last fine plane belongs to no block).  Coarse pixels likewise sit
 * at the centres of the pixel pairs they average.  Returns -1 when a
 * coarse size would be below 1. */
int or_coarse(const int *dims, const double *par, int *cdims, double *cpar)
{
    int n[5] = {dims[0], dims[1], dims[2], dims[3], dims[4]};
    for (int a = 0; a < 5; ++a)
        if (n[a] / 2 < 1) return -1;
    geom_t g = unpack(dims, par, NULL);
    cdims[0] = n[0] / 2; cdims[1] = n[1] / 2; cdims[2] = n[2] / 2;
    cdims[3] = n[3] / 2; cdims[4] = n[4] / 2; cdims[5] = dims[5];
    double h[3] = {g.hx, g.hy, g.hz};
    for (int a = 0; a < 3; ++a) cpar[a] = 2.0 * h[a];
    cpar[3] = 2.0 * g.au;
    cpar[4] = 2.0 * g.av;
    cpar[5] = g.sad;
    cpar[6] = g.sdd;
    cpar[7] = 2.0 * g.step;
    cpar[8] = g.u_off - 0.5 * g.au * (double)(n[3] & 1);
    cpar[9] = g.v_off - 0.5 * g.av * (double)(n[4] & 1);
    for (int a = 0; a < 3; ++a) cpar[10 + a] = g.off[a] - 0.5 * h[a] * (double)(n[a] & 1);
    return 0;
}

#define OR_MAX_LEVELS 4

/* Full solve with the coarse-to-fine schedule.
 *   Y: [n_views][nv][nu] fine data; f: fine volume, in = f0, out = result.
 *   n_levels 1..4; iters[level] outer iterations (coarse first), a
 *   maximum when tol > 0;
 *   beta[level] <= 0 -> 1.1*mu*(2 N_vox/N_meas)*lambda (30 power steps);
 *   n_inner[level] <= 0 -> or_default_inner.
 *   used (optional, 3 * n_levels): beta, n_inner and iterations made per
 *   level; change (optional, n_levels): relative change of each level's
 *   last iteration (tol > 0).
 *   trace (optional): rows of (E, E_eps, E1, E2), packed: (iterations
 *   made + 1) rows per level, coarse first.
 *   report (optional): E, E_eps, E1, E2 of the returned f (fine level).
 *   grad_mode 0: Step 1 with the matched transpose; 1: with Eq. (2).
 * Returns 0, or -1 on invalid sizes. */
int or_fbs_solve(const int *dims, const double *par, const double *angles,
                 const double *Y, double *f, double mu, int n_levels,
                 const int *iters, const double *beta, double eps,
                 const int *n_inner, double tol, double tv_weight, int clip_mode,
                 int grad_mode, double *used, double *change, double *trace,
                 double *report)
{
    if (n_levels < 1 || n_levels > OR_MAX_LEVELS) return -1;
    int ldims[OR_MAX_LEVELS][6];
    double lpar[OR_MAX_LEVELS][13];
    const double *lY[OR_MAX_LEVELS];
    double *lf[OR_MAX_LEVELS];
    double *owned[2 * OR_MAX_LEVELS] = {NULL};
    int fine = n_levels - 1;
    geom_t g = unpack(dims, par, angles);
    double fpar[13] = {g.hx, g.hy, g.hz, g.au, g.av, g.sad, g.sdd, g.step, g.u_off, g.v_off,
                       g.off[0], g.off[1], g.off[2]};
    memcpy(ldims[fine], dims, sizeof(int) * 6);
    memcpy(lpar[fine], fpar, sizeof(fpar));
    lY[fine] = Y;
    lf[fine] = f;
    for (int l = fine - 1; l >= 0; --l)
        if (or_coarse(ldims[l + 1], lpar[l + 1], ldims[l], lpar[l])) return -1;
    /* data and start of every coarser level from the next finer one */
    for (int l = fine - 1; l >= 0; --l) {
        const int *d = ldims[l], *D = ldims[l + 1];
        double *yc = (double *)malloc(sizeof(double) * (size_t)d[3] * d[4] * d[5]);
        double *fc = (double *)malloc(sizeof(double) * (size_t)d[0] * d[1] * d[2]);
        owned[2 * l] = yc;
        owned[2 * l + 1] = fc;
        or_bin_detector(D[3], D[4], D[5], lY[l + 1], yc);
        or_restrict(D, lf[l + 1], fc);
        lY[l] = yc;
        lf[l] = fc;
    }
    double *tr = trace;
    for (int l = 0; l < n_levels; ++l) {
        const int *d = ldims[l];
        const double *p = lpar[l];
        double h[3] = {p[0], p[1], p[2]};
        long nvox = (long)d[0] * d[1] * d[2], nmeas = (long)d[3] * d[4] * d[5];
        double b = beta ? beta[l] : 0.0;
        if (b <= 0.0)
            b = 1.1 * mu * 2.0 * (double)nvox / (double)nmeas * or_power_lambda(d, p, angles, 30);
        int k = n_inner ? n_inner[l] : 0;
        if (k <= 0) k = or_default_inner(h, b, eps);
        double ch = 0.0;
        int made = fbs_level(d, p, angles, lY[l], lf[l], mu, b, eps, k, iters[l], tol,
                             tv_weight, clip_mode, grad_mode, tr, &ch);
        if (used) {
            used[l] = b;
            used[n_levels + l] = (double)k;
            used[2 * n_levels + l] = (double)made;
        }
        if (change) change[l] = ch;
        if (tr) tr += 4 * (made + 1);
        if (l < fine) or_prolong(ldims[l], ldims[l + 1], lf[l], lf[l + 1]);
    }
    if (report) energies(dims, fpar, angles, f, Y, mu, eps, report);
    for (int q = 0; q < 2 * OR_MAX_LEVELS; ++q) free(owned[q]);
    return 0;
}

/* Number of OpenMP threads the parallel loops above use. */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
