// C ABI of the cone-beam library: plans, operators, and the forward-backward
// splitting solver of Algorithm A1 with the cascadic coarse-to-fine
// multigrid schedule (up to CBCT_MAX_LEVELS levels).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <new>
#include <string>

#include "cbct_internal.hpp"

using namespace cbct;

// ================================================================ errors ===

namespace {
thread_local std::string g_last_error;
}

namespace cbct {

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return CBCT_OK;
    return set_error(e == hipErrorOutOfMemory ? CBCT_ENOMEM : CBCT_EHIP,
                     std::string(what) + ": " + hipGetErrorString(e));
}

// ================================================================ memory ===

namespace {
std::mutex g_pool_mu;
hipMemPool_t g_pools[64] = {};
}  // namespace

static hipMemPool_t pool_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pools[dev]) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        g_pools[dev] = pool;
    }
    return g_pools[dev];
}

hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s) {
    hipMemPool_t pool = pool_for_current_device();
    if (!pool) return hipErrorOutOfMemory;
    if (bytes == 0) bytes = 256;
    return hipMallocFromPoolAsync(p, bytes, pool, s);
}

hipError_t scratch_free(void *p, hipStream_t s) {
    if (!p) return hipSuccess;
    return hipFreeAsync(p, s);
}

GridConst grid_of(const cbct_geom &g) {
    GridConst c;
    c.nx = g.nx;
    c.ny = g.ny;
    c.nz = g.nz;
    c.hx = (float)g.hx;
    c.hy = (float)g.hy;
    c.hz = (float)g.hz;
    c.x0 = (float)(-0.5 * (g.nx - 1) * g.hx + g.x_off);
    c.y0 = (float)(-0.5 * (g.ny - 1) * g.hy + g.y_off);
    c.z0 = (float)(-0.5 * (g.nz - 1) * g.hz + g.z_off);
    return c;
}

// ============================================================ timing ===
// Opt-in per-kernel device timing: when enabled, each launch made through
// timed() is bracketed by two HIP events recorded on the launch stream.

namespace {
struct TimingRec {
    int id;
    hipEvent_t a, b;
};
std::mutex g_tmu;
std::atomic<uint32_t> g_timing_mask{0};  // bit k: record kernel kind k
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_spare;

hipEvent_t take_event() {
    if (!g_spare.empty()) {
        hipEvent_t e = g_spare.back();
        g_spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

template <class F>
hipError_t timed(int id, hipStream_t s, F &&launch) {
    if (!((g_timing_mask.load(std::memory_order_relaxed) >> id) & 1u)) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        a = take_event();
        b = take_event();
    }
    if (a) (void)hipEventRecord(a, s);
    hipError_t e = launch();
    if (b) (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_tmu);
    if (a && b) g_recs.push_back({id, a, b});
    return e;
}

}  // namespace cbct

extern "C" int cbct_kernel_timing_select(uint32_t mask) {
    if (mask >> CBCT_KERNEL_COUNT) return set_error(CBCT_EINVAL, "unknown kernel kind in mask");
    std::lock_guard<std::mutex> lk(g_tmu);
    if (mask) {
        for (auto &r : g_recs) {
            g_spare.push_back(r.a);
            g_spare.push_back(r.b);
        }
        g_recs.clear();
    }
    g_timing_mask.store(mask, std::memory_order_relaxed);
    return CBCT_OK;
}

extern "C" int cbct_kernel_timing(int32_t enable) {
    return cbct_kernel_timing_select(enable ? (1u << CBCT_KERNEL_COUNT) - 1u : 0u);
}

extern "C" int cbct_kernel_timing_read(int32_t kernel, int64_t *launches, double *total_ms) {
    if (!launches || !total_ms || kernel < 0 || kernel >= CBCT_KERNEL_COUNT)
        return set_error(CBCT_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    int64_t n = 0;
    double t = 0.0;
    for (auto &r : g_recs) {
        if (r.id != kernel) continue;
        int rc = check_hip(hipEventSynchronize(r.b), "event sync");
        if (rc) return rc;
        float ms = 0.0f;
        rc = check_hip(hipEventElapsedTime(&ms, r.a, r.b), "event time");
        if (rc) return rc;
        t += ms;
        ++n;
    }
    *launches = n;
    *total_ms = t;
    return CBCT_OK;
}

extern "C" int cbct_kernel_config(int32_t *out_host, int32_t n) {
    if (!out_host || n < 0) return set_error(CBCT_EINVAL, "bad argument");
    int32_t v[8];
    projector_config(v);
    cell_pass_config(v + 4);
    for (int i = 0; i < n && i < 8; ++i) out_host[i] = v[i];
    return n < 8 ? n : 8;
}

extern "C" int cbct_probe_fma_rate(int32_t fp64, double *tflops_host, void *stream) {
    if (!tflops_host) return set_error(CBCT_EINVAL, "tflops_host is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, ncu = 0;
    int rc = check_hip(hipGetDevice(&dev), "device");
    if (!rc) rc = check_hip(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (rc) return rc;
    const int blocks = std::max(ncu, 1) * 16, iters = 8192;
    const size_t bytes = (size_t)blocks * 256 * (fp64 ? sizeof(double) : sizeof(float));
    void *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    rc = check_hip(hipMalloc(&out, bytes), "probe buffer");
    if (!rc) rc = check_hip(hipEventCreate(&a), "event");
    if (!rc) rc = check_hip(hipEventCreate(&b), "event");
    if (!rc) rc = check_hip(launch_probe_fma(fp64 != 0, out, blocks, iters, s), "probe warm-up");
    const int reps = 5;
    if (!rc) rc = check_hip(hipEventRecord(a, s), "event record");
    for (int r = 0; !rc && r < reps; ++r)
        rc = check_hip(launch_probe_fma(fp64 != 0, out, blocks, iters, s), "probe");
    if (!rc) rc = check_hip(hipEventRecord(b, s), "event record");
    if (!rc) rc = check_hip(hipEventSynchronize(b), "event sync");
    float ms = 0.0f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, a, b), "event time");
    if (!rc) {
        const double flop = (double)reps * blocks * 256.0 * iters * 8.0 * 2.0;
        *tflops_host = flop / (ms * 1e-3) / 1e12;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    return rc;
}

namespace {

// RAII holder for stream-ordered scratch.
struct Scratch {
    void *p = nullptr;
    hipStream_t s;
    explicit Scratch(hipStream_t st) : s(st) {}
    hipError_t alloc(size_t bytes) { return scratch_alloc(&p, bytes, s); }
    ~Scratch() { (void)scratch_free(p, s); }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
    void *get() const { return p; }
};

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

int validate_geom(const cbct_geom *g) {
    if (!g) return set_error(CBCT_EINVAL, "geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nu <= 0 || g->nv <= 0 || g->n_views <= 0)
        return set_error(CBCT_EINVAL, "sizes must be positive");
    if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0) || !(g->au > 0) || !(g->av > 0))
        return set_error(CBCT_EINVAL, "spacings must be positive");
    if (!(g->sad > 0) || !(g->sdd > g->sad))
        return set_error(CBCT_EINVAL, "need sdd > sad > 0");
    if (!isfinite(g->u_off) || !isfinite(g->v_off))
        return set_error(CBCT_EINVAL, "non-finite detector offset");
    if (!isfinite(g->x_off) || !isfinite(g->y_off) || !isfinite(g->z_off))
        return set_error(CBCT_EINVAL, "non-finite volume offset");
    // every corner of the zero-bordered grid stays inside the source orbit
    const double hx = 0.5 * (g->nx + 1) * g->hx + fabs(g->x_off);
    const double hy = 0.5 * (g->ny + 1) * g->hy + fabs(g->y_off);
    if (!(g->sad > sqrt(hx * hx + hy * hy)))
        return set_error(CBCT_EINVAL, "source orbit must lie outside the grid");
    const double padded = (double)(g->nx + 2) * (g->ny + 2) * (g->nz + 2);
    // float volumes are addressed with 32-bit byte offsets
    if (padded * 4.0 > 2147483647.0) return set_error(CBCT_EINVAL, "grid too large");
    if ((double)g->nu * g->nv > 2.0e9) return set_error(CBCT_EINVAL, "detector too large");
    // grid limits: views and padded planes index the third grid dimension of
    // some launches, all projector tiles form one linear grid
    if (g->n_views > 65535 || g->nz + 2 > 65535)
        return set_error(CBCT_EINVAL, "more than 65535 views or planes");
    // the transpose stores cell indices and segment numbers as 16-bit integers
    if (g->nx > 32000 || g->ny > 32000 || g->nz > 32000)
        return set_error(CBCT_EINVAL, "grid dimension above 32000");
    if ((double)project_partials_count(*g) > 2147483647.0)
        return set_error(CBCT_EINVAL, "too many detector tiles");
    if (g->angles)
        for (int k = 0; k < g->n_views; ++k)
            if (!isfinite(g->angles[k])) return set_error(CBCT_EINVAL, "non-finite angle");
    return CBCT_OK;
}

int validate_grid(const cbct_geom *g) {
    if (!g) return set_error(CBCT_EINVAL, "grid is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return set_error(CBCT_EINVAL, "sizes");
    if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0)) return set_error(CBCT_EINVAL, "spacings");
    return CBCT_OK;
}

size_t nvox_of(const cbct_geom &g) { return (size_t)g.nx * g.ny * g.nz; }
size_t nmeas_of(const cbct_geom &g) { return (size_t)g.n_views * g.nu * g.nv; }
size_t padded_of(const cbct_geom &g) { return (size_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2); }

}  // namespace

// ================================================================= plans ===

extern "C" int cbct_projector_tile_margin(const cbct_geom *g, int32_t *out_host) {
    if (!out_host) return set_error(CBCT_EINVAL, "out_host is NULL");
    const int rc = validate_geom(g);
    if (rc) return rc;
    *out_host = projector_tile_margin(*g);
    return CBCT_OK;
}

extern "C" int cbct_plan_create(const cbct_geom *gin, cbct_plan **out) {
    try {
        if (!out) return set_error(CBCT_EINVAL, "out is NULL");
        int rc = validate_geom(gin);
        if (rc) return rc;
        std::unique_ptr<cbct_plan> p(new cbct_plan());
        p->g = *gin;
        if (!(p->g.step > 0)) p->g.step = 0.5 * std::min(gin->hx, std::min(gin->hy, gin->hz));
        // sample indices n = t / step stay below (the source's distance to
        // the grid centre + half the grid diagonal) / step; keep them well
        // inside the 16-bit segment numbers of the transpose
        // (n < 32767 * 256)
        const double reach =
            std::max(p->g.sdd, p->g.sad + sqrt(pow(p->g.x_off, 2) + pow(p->g.y_off, 2) +
                                               pow(p->g.z_off, 2))) +
            0.5 * sqrt(pow((p->g.nx + 1) * p->g.hx, 2) + pow((p->g.ny + 1) * p->g.hy, 2) +
                       pow((p->g.nz + 1) * p->g.hz, 2));
        if (reach / p->g.step > 8.0e6)
            return set_error(CBCT_EINVAL, "step too small for the source distance");
        p->angles.resize(gin->n_views);
        for (int k = 0; k < gin->n_views; ++k)
            p->angles[k] = gin->angles ? gin->angles[k] : 2.0 * M_PI * k / gin->n_views;
        p->g.angles = p->angles.data();
        const cbct_geom &g = p->g;
        const double step = g.step;
        const double h[3] = {g.hx, g.hy, g.hz};
        const int n[3] = {g.nx, g.ny, g.nz};
        double x0[3];
        const double off[3] = {g.x_off, g.y_off, g.z_off};
        for (int a = 0; a < 3; ++a) x0[a] = -0.5 * (n[a] - 1) * h[a] + off[a];
        p->h_views.resize(g.n_views);
        for (int k = 0; k < g.n_views; ++k) {
            const double th = p->angles[k], cs = cos(th), sn = sin(th);
            const double src[3] = {g.sad * sn, -g.sad * cs, 0.0};
            const double ew[2] = {-sn, cs}, eu[2] = {cs, sn};
            ViewConst &v = p->h_views[k];
            memset(&v, 0, sizeof(v));
            for (int a = 0; a < 3; ++a) {
                v.Qd[a] = (src[a] - x0[a]) / h[a];
                v.Q[a] = (float)v.Qd[a];
            }
            for (int a = 0; a < 2; ++a) {
                v.Wd[a] = step / h[a] * g.sdd * ew[a];
                v.Ud[a] = step / h[a] * eu[a];
                v.W[a] = (float)v.Wd[a];
                v.U[a] = (float)v.Ud[a];
                v.src[a] = (float)src[a];
            }
            v.Vzd = step / h[2];
            v.Vz = (float)v.Vzd;
            v.cs = (float)cs;
            v.sn = (float)sn;
            v.csd = cs;
            v.snd = sn;
        }
        DetConst &d = p->det;
        d.u0d = -0.5 * (g.nu - 1) * g.au + g.u_off;
        d.v0d = -0.5 * (g.nv - 1) * g.av + g.v_off;
        d.aud = g.au;
        d.avd = g.av;
        d.sdd2d = g.sdd * g.sdd;
        d.sddd = g.sdd;
        d.u0 = (float)d.u0d;
        d.v0 = (float)d.v0d;
        d.au = (float)g.au;
        d.av = (float)g.av;
        d.sdd2 = (float)d.sdd2d;
        d.sdd = (float)g.sdd;
        p->grid = grid_of(g);
        (void)hipGetDevice(&p->device);
        rc = check_hip(hipMalloc((void **)&p->d_views, sizeof(ViewConst) * g.n_views),
                       "plan view table");
        if (rc) return rc;
        rc = check_hip(hipMemcpy(p->d_views, p->h_views.data(), sizeof(ViewConst) * g.n_views,
                                 hipMemcpyHostToDevice),
                       "plan upload");
        if (rc) {
            (void)hipFree(p->d_views);
            return rc;
        }
        unsigned long long *dcount = nullptr;
        rc = check_hip(hipMalloc((void **)&dcount, sizeof(unsigned long long)), "count");
        if (rc) {
            (void)hipFree(p->d_views);
            return rc;
        }
        rc = check_hip(hipMemset(dcount, 0, sizeof(unsigned long long)), "count init");
        unsigned long long hcount = 0;
        if (!rc) rc = check_hip(launch_count_samples(*p, dcount, nullptr), "count kernel");
        if (!rc)
            rc = check_hip(hipMemcpy(&hcount, dcount, sizeof(hcount), hipMemcpyDeviceToHost),
                           "count readback");
        (void)hipFree(dcount);
        if (rc) {
            (void)hipFree(p->d_views);
            return rc;
        }
        p->samples = (int64_t)hcount;
        *out = p.release();
        return CBCT_OK;
    } catch (const std::bad_alloc &) {
        return set_error(CBCT_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

extern "C" void cbct_plan_destroy(cbct_plan *p) {
    if (!p) return;
    if (p->coarse) cbct_plan_destroy(p->coarse);
    if (p->bp_ready) {
        (void)hipEventSynchronize(p->bp_ready);
        (void)hipEventDestroy(p->bp_ready);
    }
    if (p->bp_geom) (void)hipFree(p->bp_geom);
    if (p->d_views) (void)hipFree(p->d_views);
    delete p;
}

extern "C" int64_t cbct_plan_samples(const cbct_plan *p) { return p ? p->samples : -1; }

extern "C" int cbct_plan_geom(const cbct_plan *p, cbct_geom *out) {
    if (!p || !out) return set_error(CBCT_EINVAL, "NULL argument");
    *out = p->g;
    return CBCT_OK;
}

// ============================================================= operators ===

namespace {

template <typename T>
int project_impl(const cbct_plan *p, const T *f, const T *Y, T *out, double *sumsq,
                 hipStream_t s) {
    if (!p || !f || !out) return set_error(CBCT_EINVAL, "NULL argument");
    Scratch pad(s), part(s);
    int rc = check_hip(pad.alloc(sizeof(T) * padded_count(*p)), "scratch (padded volume)");
    if (rc) return rc;
    const size_t np = project_partials_count(*p);
    if (sumsq) {
        rc = check_hip(part.alloc(sizeof(double) * np), "scratch (partials)");
        if (rc) return rc;
    }
    rc = check_hip(timed(CBCT_KERNEL_PAD, s, [&] { return launch_pad<T>(*p, f, pad.as<T>(), s); }), "pad kernel");
    if (rc) return rc;
    rc = check_hip(timed(CBCT_KERNEL_PROJECT, s, [&] { return launch_project<T>(*p, pad.as<T>(), Y, out, sumsq ? part.as<double>() : nullptr,
                                     s); }),
                   "project kernel");
    if (rc) return rc;
    if (sumsq) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_reduce_sum(part.as<double>(), (int)np, sumsq, 1, s); }), "reduce");
    return rc;
}

// The plan's transpose geometry tables, prepared on the first call (on
// stream s) and afterwards only waited for on s.
int plan_bp_geometry(const cbct_plan *p, hipStream_t s, const void **out) {
    std::lock_guard<std::mutex> lk(p->bp_mu);
    if (!p->bp_geom) {
        void *g = nullptr;
        int rc = check_hip(hipMalloc(&g, bp_geom_bytes(p->g)), "plan transpose tables");
        if (rc) return rc;
        hipEvent_t ev = nullptr;
        rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_bp_prepare(*p, g, s); }),
                       "ray table");
        if (!rc) rc = check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
        if (!rc) rc = check_hip(hipEventRecord(ev, s), "event record");
        if (rc) {
            if (ev) (void)hipEventDestroy(ev);
            (void)hipStreamSynchronize(s);
            (void)hipFree(g);
            return rc;
        }
        p->bp_geom = g;
        p->bp_ready = ev;
    } else {
        int rc = check_hip(hipStreamWaitEvent(s, p->bp_ready, 0), "wait for the plan tables");
        if (rc) return rc;
    }
    *out = p->bp_geom;
    return CBCT_OK;
}

template <typename T>
int backproject_impl(const cbct_plan *p, const T *y, const T *f, double tau, T *out,
                     hipStream_t s) {
    if (!p || !y || !out) return set_error(CBCT_EINVAL, "NULL argument");
    const void *geom = nullptr;
    int rc = plan_bp_geometry(p, s, &geom);
    if (rc) return rc;
    Scratch cells(s);
    rc = check_hip(cells.alloc(bp_cells_bytes(p->g, sizeof(T))), "scratch (transpose cell sums)");
    if (rc) return rc;
    rc = check_hip(timed(CBCT_KERNEL_CELLS, s, [&] { return launch_backproject_cells<T>(*p, y, cells.get(), geom, s); }), "cell kernel");
    if (rc) return rc;
    return check_hip(timed(CBCT_KERNEL_GATHER, s, [&] { return launch_gather_cells<T>(*p, cells.get(), f, tau, out, s); }), "gather kernel");
}

}  // namespace

extern "C" int cbct_project(const cbct_plan *p, const float *f, float *y, void *stream) {
    return project_impl<float>(p, f, nullptr, y, nullptr, as_stream(stream));
}

extern "C" int cbct_project_residual(const cbct_plan *p, const float *f, const float *Y,
                                     float *r, double *sumsq, void *stream) {
    if (!Y) return set_error(CBCT_EINVAL, "Y is NULL");
    return project_impl<float>(p, f, Y, r, sumsq, as_stream(stream));
}

extern "C" int cbct_backproject(const cbct_plan *p, const float *y, float *f, void *stream) {
    return backproject_impl<float>(p, y, nullptr, 0.0, f, as_stream(stream));
}

extern "C" int cbct_backproject_update(const cbct_plan *p, const float *r, const float *f,
                                       double tau, float *g, void *stream) {
    if (!f) return set_error(CBCT_EINVAL, "f is NULL");
    if (!isfinite(tau)) return set_error(CBCT_EINVAL, "tau not finite");
    return backproject_impl<float>(p, r, f, tau, g, as_stream(stream));
}

extern "C" int cbct_backproject_eq2(const cbct_plan *p, const float *y, float *f,
                                    void *stream) {
    if (!p || !y || !f) return set_error(CBCT_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    return check_hip(timed(CBCT_KERNEL_EQ2, s, [&] { return launch_eq2(*p, y, nullptr, 0.0, f, s); }),
                     "eq2 kernel");
}

extern "C" int cbct_log_counts(const float *counts, const float *flat, double i0,
                               double min_count, float *y, int64_t n, void *stream) {
    if (!counts || !y) return set_error(CBCT_EINVAL, "NULL argument");
    if (n < 0 || (double)n > 1.0e15) return set_error(CBCT_EINVAL, "bad element count");
    if (!(min_count > 0) || !isfinite(min_count)) return set_error(CBCT_EINVAL, "min_count must be > 0");
    if (!flat && (!(i0 > 0) || !isfinite(i0))) return set_error(CBCT_EINVAL, "i0 must be > 0");
    hipStream_t s = as_stream(stream);
    return check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_log_counts(counts, flat, i0, min_count, y, (long long)n, s); }),
                     "log counts");
}

extern "C" int cbct_project_f64(const cbct_plan *p, const double *f, double *y, void *stream) {
    return project_impl<double>(p, f, nullptr, y, nullptr, as_stream(stream));
}

extern "C" int cbct_backproject_f64(const cbct_plan *p, const double *y, double *f,
                                    void *stream) {
    return backproject_impl<double>(p, y, nullptr, 0.0, f, as_stream(stream));
}

// ==================================================================== TV ===

namespace {

double default_prox_step(const cbct_geom &g, double beta, double eps) {
    const double d2 = 4.0 * (1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz));
    return 1.0 / (beta + d2 / eps);
}

int default_inner(const cbct_geom &g, double beta, double eps) {
    const double d2 = 4.0 * (1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz));
    const double k = ceil(3.0 * (1.0 + d2 / (eps * beta)));
    return k > 200.0 ? 200 : (int)k;
}

// K sweeps from z0 = f (in place), ping-ponging with `tmp` (nvox floats).
// `timing` = false launches without the diagnostic HIP events (whose
// creation the no-allocation entry point must not make).
int prox_sweeps(const GridConst &gc, size_t nvox, const float *g, float *f, float *tmp,
                double beta, double eps, int n_inner, double step, int nonneg, hipStream_t s,
                bool timing = true) {
    float *a = f, *b = tmp;
    for (int m = 0; m < n_inner; ++m) {
        auto launch = [&] {
            return launch_tv_sweep(gc, a, g, b, (float)beta, (float)eps, (float)step, nonneg, s);
        };
        int rc = check_hip(timing ? timed(CBCT_KERNEL_TV_SWEEP, s, launch) : launch(),
                           "tv sweep");
        if (rc) return rc;
        std::swap(a, b);
    }
    if (a != f)
        return check_hip(hipMemcpyAsync(f, a, sizeof(float) * nvox, hipMemcpyDeviceToDevice, s),
                         "prox copy");
    return CBCT_OK;
}

// E1 pieces of z into dev_out[0..1] (sum |Dz|, sum |Dz|_eps); partials
// must hold tv_energy_partials_count doubles.
int tv_sums(const GridConst &gc, const float *z, double eps, double *partials, double *dev_out,
            hipStream_t s) {
    int np = 0;
    int rc = check_hip(timed(CBCT_KERNEL_TV_ENERGY, s, [&] { return launch_tv_energy(gc, z, eps, partials, &np, s); }), "tv energy");
    if (rc) return rc;
    return check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_reduce_sum(partials, np, dev_out, 2, s); }), "reduce");
}

}  // namespace

extern "C" int cbct_tv_prox(const cbct_geom *grid, const float *g, float *f, double beta,
                            double eps, int32_t n_inner, double step, int32_t nonneg,
                            void *stream) {
    try {
        int rc = validate_grid(grid);
        if (rc) return rc;
        if (!g || !f) return set_error(CBCT_EINVAL, "NULL argument");
        if (!(beta > 0) || !(eps > 0) || n_inner < 0 || !isfinite(beta) || !isfinite(eps))
            return set_error(CBCT_EINVAL, "need beta > 0, eps > 0, n_inner >= 0");
        if (n_inner == 0) return CBCT_OK;
        if (!(step > 0)) step = default_prox_step(*grid, beta, eps);
        hipStream_t s = as_stream(stream);
        const size_t nvox = nvox_of(*grid);
        Scratch tmp(s);
        rc = check_hip(tmp.alloc(sizeof(float) * nvox), "scratch (prox)");
        if (rc) return rc;
        return prox_sweeps(grid_of(*grid), nvox, g, f, tmp.as<float>(), beta, eps, n_inner, step,
                           nonneg, s);
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

// ------------------------------------------- no-allocation TV prox ---
// The ping-pong volume of cbct_tv_prox_noalloc lives in this fixed device
// array, one copy per GPU.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in): it looks up the
// device address once per device with hipGetSymbolAddress and uses that.
constexpr size_t NOALLOC_MAX_VOXELS = size_t(1) << 24;  // 64 MiB of float

static __device__ __align__(256) float scratch[NOALLOC_MAX_VOXELS];

namespace {
std::mutex g_scratch_mu;
float *g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device.  EHIP if the lookup fails.
int scratch_address(float **out) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "current device");
    if (rc) return rc;
    if (dev < 0 || dev >= 64) return set_error(CBCT_EHIP, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (rc) return rc;
        g_scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return CBCT_OK;
}
}  // namespace

extern "C" int cbct_tv_prox_noalloc(const cbct_geom *grid, const float *g, float *f,
                                    double beta, double eps, int32_t n_inner, double step,
                                    int32_t nonneg, void *stream) {
    try {
        int rc = validate_grid(grid);
        if (rc) return rc;
        if (!g || !f) return set_error(CBCT_EINVAL, "NULL argument");
        if (!(beta > 0) || !(eps > 0) || n_inner < 0 || !isfinite(beta) || !isfinite(eps))
            return set_error(CBCT_EINVAL, "need beta > 0, eps > 0, n_inner >= 0");
        const size_t nvox = nvox_of(*grid);
        if (nvox > NOALLOC_MAX_VOXELS)
            return set_error(CBCT_EINVAL, "cbct_tv_prox_noalloc: grid of " +
                                              std::to_string(nvox) +
                                              " voxels exceeds its fixed scratch of " +
                                              std::to_string(NOALLOC_MAX_VOXELS) +
                                              " voxels; use cbct_tv_prox");
        float *tmp = nullptr;
        rc = scratch_address(&tmp);
        if (rc) return rc;
        if (n_inner == 0) return CBCT_OK;
        if (!(step > 0)) step = default_prox_step(*grid, beta, eps);
        return prox_sweeps(grid_of(*grid), nvox, g, f, tmp, beta, eps, n_inner, step, nonneg,
                           as_stream(stream), false);
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

extern "C" int cbct_tv_energy(const cbct_geom *grid, const float *f, double eps,
                              double *out_host, void *stream) {
    int rc = validate_grid(grid);
    if (rc) return rc;
    if (!f || !out_host) return set_error(CBCT_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    const GridConst gc = grid_of(*grid);
    Scratch part(s), res(s);
    rc = check_hip(part.alloc(sizeof(double) * tv_energy_partials_count(gc)), "scratch");
    if (rc) return rc;
    rc = check_hip(res.alloc(sizeof(double) * 2), "scratch");
    if (rc) return rc;
    rc = tv_sums(gc, f, eps, part.as<double>(), res.as<double>(), s);
    if (rc) return rc;
    double h[2];
    rc = check_hip(hipMemcpyAsync(h, res.p, sizeof(h), hipMemcpyDeviceToHost, s), "readback");
    if (rc) return rc;
    rc = check_hip(hipStreamSynchronize(s), "sync");
    if (rc) return rc;
    const double n = (double)nvox_of(*grid);
    out_host[0] = h[0] / n;
    out_host[1] = h[1] / n;
    return CBCT_OK;
}

// ====================================================== power iteration ===

extern "C" int cbct_plan_lambda(const cbct_plan *p, int32_t n_iter, double *lambda_host,
                                void *stream) {
    try {
        if (!p || !lambda_host || n_iter <= 0) return set_error(CBCT_EINVAL, "bad argument");
        {
            std::lock_guard<std::mutex> lk(p->lam_mu);
            for (auto &e : p->lam_cache)
                if (e.first == n_iter) {
                    *lambda_host = e.second;
                    return CBCT_OK;
                }
        }
        hipStream_t s = as_stream(stream);
        const size_t nvox = nvox_of(p->g), nmeas = nmeas_of(p->g);
        Scratch x(s), y(s), w(s), pad(s), cells(s), part(s), sc(s);
        int rc = check_hip(x.alloc(sizeof(float) * nvox), "scratch");
        if (!rc) rc = check_hip(y.alloc(sizeof(float) * nmeas), "scratch");
        if (!rc) rc = check_hip(w.alloc(sizeof(float) * nvox), "scratch");
        if (!rc) rc = check_hip(pad.alloc(sizeof(float) * padded_count(*p)), "scratch");
        if (!rc) rc = check_hip(cells.alloc(bp_workspace_bytes(p->g, sizeof(float))), "scratch");
        if (!rc) rc = check_hip(part.alloc(sizeof(double) * 4096), "scratch");
        if (!rc) rc = check_hip(sc.alloc(sizeof(double)), "scratch");
        if (rc) return rc;
        rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_fill(x.as<float>(), nvox, (float)(1.0 / sqrt((double)nvox)), s); }),
                       "fill");
        if (!rc) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_bp_prepare(*p, bp_geom_in(cells.get(), p->g, sizeof(float)), s); }), "ray table");
        for (int it = 0; !rc && it < n_iter; ++it) {
            rc = check_hip(timed(CBCT_KERNEL_PAD, s, [&] { return launch_pad<float>(*p, x.as<float>(), pad.as<float>(), s); }), "pad");
            if (!rc)
                rc = check_hip(timed(CBCT_KERNEL_PROJECT, s, [&] { return launch_project<float>(*p, pad.as<float>(), nullptr, y.as<float>(),
                                                     nullptr, s); }),
                               "project");
            if (!rc)
                rc = check_hip(timed(CBCT_KERNEL_CELLS, s, [&] { return launch_backproject_cells<float>(*p, y.as<float>(), cells.get(),
                                                               bp_geom_in(cells.get(), p->g, sizeof(float)), s); }),
                               "cells");
            if (!rc)
                rc = check_hip(timed(CBCT_KERNEL_GATHER, s, [&] { return launch_gather_cells<float>(*p, cells.get(), nullptr, 0.0,
                                                          w.as<float>(), s); }),
                               "gather");
            int np = 0;
            if (!rc) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_sumsq(w.as<float>(), nvox, part.as<double>(), &np, s); }), "sumsq");
            if (!rc) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_reduce_sum(part.as<double>(), np, sc.as<double>(), 1, s); }), "reduce");
            if (!rc) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_scale(w.as<float>(), nvox, sc.as<double>(), x.as<float>(), s); }), "scale");
        }
        if (rc) return rc;
        double n2 = 0.0;
        rc = check_hip(hipMemcpyAsync(&n2, sc.p, sizeof(double), hipMemcpyDeviceToHost, s), "readback");
        if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync");
        if (rc) return rc;
        const double lam = sqrt(n2);
        {
            std::lock_guard<std::mutex> lk(p->lam_mu);
            p->lam_cache.emplace_back(n_iter, lam);
        }
        *lambda_host = lam;
        return CBCT_OK;
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

// ================================================================= solver ===

namespace {

struct Level {
    const cbct_plan *plan = nullptr;
    const float *Y = nullptr;
    float *f = nullptr;
    float *g = nullptr, *z = nullptr, *r = nullptr, *pad = nullptr, *cells = nullptr;
    float *fprev = nullptr;  // f before the outer iteration (tol > 0)
    double beta = 0, tau = 0, prox_step = 0;
    int n_inner = 0, iters = 0;
    int made = 0;            // outer iterations made
    double change = 0;       // relative change of the last one (tol > 0)
    bool stopped = false;    // the tolerance was met
    size_t nvox = 0, nmeas = 0;
};

}  // namespace

struct cbct_fbs_state {
    Level lv[CBCT_MAX_LEVELS];
    int n_levels = 1;
    int level = 0, iter = 0;
    bool done = false;
    cbct_fbs_params prm;
    double *partials = nullptr;  // max of the per-level partial counts
    double *dsc = nullptr;       // device scalars [4]
    std::vector<void *> owned;   // stream-ordered allocations
    std::vector<double> trace;   // rows of (E, E_eps, E1, E2)
    double final_e[4] = {0, 0, 0, 0};
    bool have_final = false;
    hipStream_t last_stream = nullptr;
};

namespace {

// The next coarser level: a coarse cell averages fine voxels (2i, 2i + 1)
// along each axis and sits at their centre, so an odd axis moves the
// coarse grid's centre half a fine spacing down; pixels likewise.
cbct_geom coarse_geom(const cbct_geom &g) {
    cbct_geom c = g;
    c.x_off = g.x_off - 0.5 * g.hx * (double)(g.nx & 1);
    c.y_off = g.y_off - 0.5 * g.hy * (double)(g.ny & 1);
    c.z_off = g.z_off - 0.5 * g.hz * (double)(g.nz & 1);
    c.u_off = g.u_off - 0.5 * g.au * (double)(g.nu & 1);
    c.v_off = g.v_off - 0.5 * g.av * (double)(g.nv & 1);
    c.nx = g.nx / 2;
    c.ny = g.ny / 2;
    c.nz = g.nz / 2;
    c.hx = 2 * g.hx;
    c.hy = 2 * g.hy;
    c.hz = 2 * g.hz;
    c.nu = g.nu / 2;
    c.nv = g.nv / 2;
    c.au = 2 * g.au;
    c.av = 2 * g.av;
    c.step = 2 * g.step;
    return c;
}

int validate_params(const cbct_geom &g, const cbct_fbs_params *prm) {
    if (!prm) return set_error(CBCT_EINVAL, "params NULL");
    if (prm->n_levels < 1 || prm->n_levels > CBCT_MAX_LEVELS)
        return set_error(CBCT_EINVAL, "n_levels must be 1 to CBCT_MAX_LEVELS");
    if (!(prm->mu > 0) || !isfinite(prm->mu)) return set_error(CBCT_EINVAL, "mu must be > 0");
    if (!(prm->eps > 0) || !isfinite(prm->eps)) return set_error(CBCT_EINVAL, "eps must be > 0");
    for (int l = 0; l < prm->n_levels; ++l) {
        if (prm->iters[l] < 0) return set_error(CBCT_EINVAL, "iters must be >= 0");
        if (!isfinite(prm->beta[l])) return set_error(CBCT_EINVAL, "beta not finite");
    }
    if (!(prm->tol >= 0) || !isfinite(prm->tol)) return set_error(CBCT_EINVAL, "tol must be >= 0");
    cbct_geom c = g;
    for (int l = 1; l < prm->n_levels; ++l) {
        if (c.nx < 2 || c.ny < 2 || c.nz < 2 || c.nu < 2 || c.nv < 2)
            return set_error(CBCT_EINVAL, "a coarser level would have a size below 1");
        c = coarse_geom(c);
        // the coarser plan must be creatable too (its padded grid is larger)
        const int rc = validate_geom(&c);
        if (rc) return rc;
    }
    if (prm->gradient != 0 && prm->gradient != 1)
        return set_error(CBCT_EINVAL, "gradient must be 0 (transpose) or 1 (Eq. (2))");
    if (prm->trace_energy < 0 || prm->trace_energy > 2)
        return set_error(CBCT_EINVAL, "trace_energy must be 0, 1 or 2");
    return CBCT_OK;
}

// Device bytes of one level's state; the Eq. (2) gradient needs no
// transpose workspace.
size_t level_bytes(const cbct_geom &g, bool own_yf, int gradient, bool tol) {
    const size_t nvox = nvox_of(g), nmeas = nmeas_of(g);
    size_t b = sizeof(float) * (2 * nvox + nmeas + padded_of(g));
    if (gradient == 0) b += bp_workspace_bytes(g, sizeof(float));
    if (tol) b += sizeof(float) * nvox;
    if (own_yf) b += sizeof(float) * (nvox + nmeas);
    return b;
}

size_t partials_needed(const cbct_plan &p) {
    return std::max(project_partials_count(p), tv_energy_partials_count(p.grid));
}

int alloc_owned(cbct_fbs_state *st, void **p, size_t bytes, hipStream_t s) {
    int rc = check_hip(scratch_alloc(p, bytes, s), "solver state allocation");
    if (!rc) st->owned.push_back(*p);
    return rc;
}

// r = P f - Y for the level's current f; with `energy`, also the energies
// of f into row (E, E_eps, E1, E2), which syncs the stream.
int level_residual(cbct_fbs_state *st, Level &L, hipStream_t s, bool energy, double row[4]) {
    const cbct_plan &p = *L.plan;
    int rc = check_hip(timed(CBCT_KERNEL_PAD, s, [&] { return launch_pad<float>(p, L.f, L.pad, s); }), "pad");
    if (!rc)
        rc = check_hip(timed(CBCT_KERNEL_PROJECT, s, [&] {
                           return launch_project<float>(p, L.pad, L.Y, L.r,
                                                        energy ? st->partials : nullptr, s);
                       }),
                       "project");
    if (rc || !energy) return rc;
    rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] {
                       return launch_reduce_sum(st->partials, (int)project_partials_count(p),
                                                st->dsc, 1, s);
                   }),
                   "reduce");
    if (!rc) rc = tv_sums(p.grid, L.f, st->prm.eps, st->partials, st->dsc + 1, s);
    if (rc) return rc;
    double h[3];
    rc = check_hip(hipMemcpyAsync(h, st->dsc, sizeof(h), hipMemcpyDeviceToHost, s), "readback");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync");
    if (rc) return rc;
    const double e2 = h[0] / (double)L.nmeas;
    const double e1 = h[1] / (double)L.nvox, e1e = h[2] / (double)L.nvox;
    row[0] = e1 + st->prm.mu * e2;
    row[1] = e1e + st->prm.mu * e2;
    row[2] = e1;
    row[3] = e2;
    if (!isfinite(row[0]) || !isfinite(row[1]))
        return set_error(CBCT_ENONFINITE, "non-finite energy");
    return CBCT_OK;
}

// One outer iteration of Algorithm A1 on level L (the residual r = P f - Y
// is already in L.r when have_residual).
int fbs_iteration(cbct_fbs_state *st, Level &L, hipStream_t s, bool have_residual) {
    const cbct_plan &p = *L.plan;
    // Step 1 (update): r = P f - Y, g = f - tau P^T r
    int rc = have_residual ? CBCT_OK : level_residual(st, L, s, false, nullptr);
    if (st->prm.gradient == 1) {
        // the paper's Eq. (2) as printed, fused with the update
        if (!rc) rc = check_hip(timed(CBCT_KERNEL_EQ2, s, [&] { return launch_eq2(p, L.r, L.f, L.tau, L.g, s); }), "eq2");
    } else {
        if (!rc) rc = check_hip(timed(CBCT_KERNEL_CELLS, s, [&] { return launch_backproject_cells<float>(p, L.r, L.cells, bp_geom_in(L.cells, p.g, sizeof(float)), s); }), "cells");
        if (!rc) rc = check_hip(timed(CBCT_KERNEL_GATHER, s, [&] { return launch_gather_cells<float>(p, L.cells, L.f, L.tau, L.g, s); }), "gather");
    }
    // Steps 2 and 3 (minimise, correct), from z0 = f
    if (!rc)
        rc = prox_sweeps(p.grid, L.nvox, L.g, L.f, L.z, L.beta, st->prm.eps, L.n_inner,
                         L.prox_step, 1, s);
    return rc;
}

// Relative change ||f - fprev|| / ||f|| of the outer iteration just made
// (0 when both are zero, +inf when only f is); syncs the stream.
int level_change(cbct_fbs_state *st, Level &L, hipStream_t s, double *out) {
    int np = 0;
    int rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_diff_sums(L.f, L.fprev, L.nvox, st->partials, &np, s); }),
                       "change sums");
    if (!rc)
        rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_reduce_sum(st->partials, np, st->dsc, 2, s); }),
                       "reduce");
    double h[2] = {0, 0};
    if (!rc) rc = check_hip(hipMemcpyAsync(h, st->dsc, sizeof(h), hipMemcpyDeviceToHost, s), "readback");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync");
    if (rc) return rc;
    *out = h[1] > 0 ? sqrt(h[0] / h[1]) : (h[0] > 0 ? INFINITY : 0.0);
    return CBCT_OK;
}

}  // namespace

extern "C" size_t cbct_fbs_footprint(const cbct_geom *g, const cbct_fbs_params *prm) {
    if (validate_geom(g) || validate_params(*g, prm)) return 0;
    size_t b = sizeof(float) * (nvox_of(*g) + nmeas_of(*g));  // caller's f and Y
    const bool tol = prm->tol > 0;
    b += level_bytes(*g, false, prm->gradient, tol);
    cbct_geom c = *g;
    for (int l = 1; l < prm->n_levels; ++l) {
        c = coarse_geom(c);
        b += level_bytes(c, true, prm->gradient, tol);
    }
    // partials and scalars
    size_t np = std::max(project_partials_count(*g),
                         (size_t)2 * ((g->nx + 63) / 64) * ((g->ny + 3) / 4) * g->nz);
    if (tol) np = std::max(np, (size_t)2 * DIFF_BLOCKS);
    b += sizeof(double) * (np + 8);
    // beta from the power iteration: cbct_plan_lambda's scratch for the
    // finest level, held during init (counted even when the plan has the
    // estimate cached already)
    bool estimate = false;
    for (int l = 0; l < prm->n_levels; ++l) estimate |= !(prm->beta[l] > 0);
    if (estimate)
        b += sizeof(float) * (2 * nvox_of(*g) + nmeas_of(*g) + padded_of(*g)) +
             bp_workspace_bytes(*g, sizeof(float)) + sizeof(double) * (4096 + 1);
    return b;
}

extern "C" int cbct_fbs_init(const cbct_plan *fine, const float *Y, float *f,
                             const cbct_fbs_params *prm, cbct_fbs_state **out, void *stream) {
    try {
        if (!fine || !Y || !f || !out) return set_error(CBCT_EINVAL, "NULL argument");
        int rc = validate_params(fine->g, prm);
        if (rc) return rc;
        hipStream_t s = as_stream(stream);
        std::unique_ptr<cbct_fbs_state> st(new cbct_fbs_state());
        st->prm = *prm;
        st->n_levels = prm->n_levels;
        st->last_stream = s;
        const int fi = prm->n_levels - 1;
        st->lv[fi].plan = fine;
        st->lv[fi].Y = Y;
        st->lv[fi].f = f;
        // the chain of coarser plans, each cached in the next finer one
        for (int l = fi - 1; l >= 0; --l) {
            const cbct_plan *up = st->lv[l + 1].plan;
            std::lock_guard<std::mutex> lk(up->coarse_mu);
            if (!up->coarse) {
                cbct_geom cg = coarse_geom(up->g);
                cg.angles = up->angles.data();
                cbct_plan *cp = nullptr;
                rc = cbct_plan_create(&cg, &cp);
                if (rc) return rc;
                up->coarse = cp;
            }
            st->lv[l].plan = up->coarse;
        }
        const bool tol = prm->tol > 0;
        size_t np = tol ? (size_t)2 * DIFF_BLOCKS : 8;
        for (int l = 0; l < st->n_levels; ++l) {
            Level &L = st->lv[l];
            const cbct_geom &g = L.plan->g;
            L.nvox = nvox_of(g);
            L.nmeas = nmeas_of(g);
            np = std::max(np, partials_needed(*L.plan));
        }
        auto cleanup = [&]() {
            for (void *p : st->owned) (void)scratch_free(p, s);
            st->owned.clear();
        };
        rc = alloc_owned(st.get(), (void **)&st->partials, sizeof(double) * np, s);
        if (!rc) rc = alloc_owned(st.get(), (void **)&st->dsc, sizeof(double) * 8, s);
        for (int l = 0; !rc && l < st->n_levels; ++l) {
            Level &L = st->lv[l];
            const cbct_plan &p = *L.plan;
            if (l < fi) {
                rc = alloc_owned(st.get(), (void **)&L.f, sizeof(float) * L.nvox, s);
                if (!rc) rc = alloc_owned(st.get(), (void **)&L.Y, sizeof(float) * L.nmeas, s);
            }
            if (!rc) rc = alloc_owned(st.get(), (void **)&L.g, sizeof(float) * L.nvox, s);
            if (!rc) rc = alloc_owned(st.get(), (void **)&L.z, sizeof(float) * L.nvox, s);
            if (!rc) rc = alloc_owned(st.get(), (void **)&L.r, sizeof(float) * L.nmeas, s);
            if (!rc) rc = alloc_owned(st.get(), (void **)&L.pad, sizeof(float) * padded_count(p), s);
            if (!rc && tol) rc = alloc_owned(st.get(), (void **)&L.fprev, sizeof(float) * L.nvox, s);
            if (!rc && prm->gradient == 0) {
                rc = alloc_owned(st.get(), (void **)&L.cells, bp_workspace_bytes(p.g, sizeof(float)), s);
                if (!rc) rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_bp_prepare(p, bp_geom_in(L.cells, p.g, sizeof(float)), s); }), "ray table");
            }
        }
        // data and start of each coarser level from the next finer one
        for (int l = fi - 1; !rc && l >= 0; --l) {
            const Level &U = st->lv[l + 1];
            Level &L = st->lv[l];
            const cbct_geom &g = U.plan->g;
            rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_bin_detector(U.Y, g.nu, g.nv, g.n_views, (float *)L.Y, s); }),
                           "bin detector");
            if (!rc)
                rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_restrict(U.f, g.nx, g.ny, g.nz, L.f, s); }), "restrict");
        }
        // beta, tau, inner count per level
        for (int l = 0; !rc && l < st->n_levels; ++l) {
            Level &L = st->lv[l];
            const cbct_geom &g = L.plan->g;
            double beta = prm->beta[l];
            if (!(beta > 0)) {
                double lam = 0;
                rc = cbct_plan_lambda(L.plan, 30, &lam, stream);
                if (rc) break;
                beta = 1.1 * prm->mu * 2.0 * (double)L.nvox / (double)L.nmeas * lam;
                if (!(beta > 0) || !isfinite(beta)) {
                    rc = set_error(CBCT_EINVAL, "beta estimate not positive");
                    break;
                }
            }
            L.beta = beta;
            L.tau = (prm->mu / beta) * 2.0 * (double)L.nvox / (double)L.nmeas;
            L.n_inner = prm->n_inner[l] > 0 ? prm->n_inner[l] : default_inner(g, beta, prm->eps);
            L.prox_step = default_prox_step(g, beta, prm->eps);
            L.iters = prm->iters[l];
        }
        if (rc) {
            cleanup();
            return rc;
        }
        st->level = 0;
        st->iter = 0;
        st->done = false;
        *out = st.release();
        return CBCT_OK;
    } catch (const std::bad_alloc &) {
        return set_error(CBCT_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

extern "C" int cbct_fbs_step(cbct_fbs_state *st, int32_t n_iters, void *stream) {
    try {
        if (!st || n_iters < 0) return set_error(CBCT_EINVAL, "bad argument");
        hipStream_t s = as_stream(stream);
        st->last_stream = s;
        int rc = CBCT_OK;
        int left = n_iters;
        while (!st->done && !rc) {
            Level &L = st->lv[st->level];
            if (st->iter < L.iters && !L.stopped) {
                if (left == 0) break;
                const bool tr = st->prm.trace_energy == 1;
                if (tr) {
                    double row[4];
                    rc = level_residual(st, L, s, true, row);
                    if (rc) break;
                    st->trace.insert(st->trace.end(), row, row + 4);
                }
                if (L.fprev)
                    rc = check_hip(hipMemcpyAsync(L.fprev, L.f, sizeof(float) * L.nvox,
                                                  hipMemcpyDeviceToDevice, s),
                                   "keep f");
                if (!rc) rc = fbs_iteration(st, L, s, tr);
                if (rc) break;
                ++st->iter;
                L.made = st->iter;
                --left;
                if (L.fprev) {
                    rc = level_change(st, L, s, &L.change);
                    if (!rc && L.change <= st->prm.tol) L.stopped = true;
                }
                continue;
            }
            // level finished: its energy when traced, the returned volume's
            // energy also when only that is asked for
            const bool last = st->level == st->n_levels - 1;
            if (st->prm.trace_energy == 1 || (st->prm.trace_energy == 2 && last)) {
                double row[4];
                rc = level_residual(st, L, s, true, row);
                if (rc) break;
                if (st->prm.trace_energy == 1) st->trace.insert(st->trace.end(), row, row + 4);
                if (last) {
                    memcpy(st->final_e, row, sizeof(row));
                    st->have_final = true;
                }
            }
            if (st->level + 1 < st->n_levels) {
                Level &F = st->lv[st->level + 1];
                const cbct_geom &cg = L.plan->g, &fg = F.plan->g;
                rc = check_hip(timed(CBCT_KERNEL_OTHER, s, [&] { return launch_prolong(L.f, cg.nx, cg.ny, cg.nz, F.f, fg.nx, fg.ny, fg.nz, s); }),
                               "prolong");
                ++st->level;
                st->iter = 0;
            } else {
                st->done = true;
            }
        }
        return rc;
    } catch (...) {
        return set_error(CBCT_EHIP, "unexpected exception");
    }
}

extern "C" int cbct_fbs_finished(const cbct_fbs_state *st) {
    if (!st) return set_error(CBCT_EINVAL, "NULL state");
    return st->done ? 1 : 0;
}

extern "C" int cbct_fbs_report_get(const cbct_fbs_state *st, cbct_fbs_report *rep) {
    if (!st || !rep) return set_error(CBCT_EINVAL, "NULL argument");
    rep->E = st->have_final ? st->final_e[0] : 0.0;
    rep->E_eps = st->have_final ? st->final_e[1] : 0.0;
    rep->E1 = st->have_final ? st->final_e[2] : 0.0;
    rep->E2 = st->have_final ? st->final_e[3] : 0.0;
    int done = 0;
    for (int l = 0; l < CBCT_MAX_LEVELS; ++l) {
        const bool in = l < st->n_levels;
        rep->beta_used[l] = in ? st->lv[l].beta : 0.0;
        rep->n_inner_used[l] = in ? st->lv[l].n_inner : 0;
        rep->level_iters[l] = in ? st->lv[l].made : 0;
        rep->change[l] = in ? st->lv[l].change : 0.0;
        done += rep->level_iters[l];
    }
    rep->iters_done = done;
    if (rep->trace && !st->trace.empty())
        memcpy(rep->trace, st->trace.data(), sizeof(double) * st->trace.size());
    return CBCT_OK;
}

extern "C" void cbct_fbs_free(cbct_fbs_state *st) {
    if (!st) return;
    for (void *p : st->owned) (void)scratch_free(p, st->last_stream);
    delete st;
}

extern "C" int cbct_fbs_solve(const cbct_plan *fine, const float *Y, float *f,
                              const cbct_fbs_params *prm, cbct_fbs_report *rep, void *stream) {
    cbct_fbs_state *st = nullptr;
    int rc = cbct_fbs_init(fine, Y, f, prm, &st, stream);
    if (rc) return rc;
    rc = cbct_fbs_step(st, INT32_MAX, stream);
    if (!rc && rep) rc = cbct_fbs_report_get(st, rep);
    cbct_fbs_free(st);
    return rc;
}

// ================================================================= misc ===

extern "C" const char *cbct_strerror(int code) {
    switch (code) {
        case CBCT_OK: return "success";
        case CBCT_EINVAL: return "invalid argument";
        case CBCT_ENOMEM: return "out of memory";
        case CBCT_EHIP: return "HIP runtime error";
        case CBCT_ENONFINITE: return "non-finite energy";
        default: return "unknown error";
    }
}

extern "C" const char *cbct_last_error(void) { return g_last_error.c_str(); }
