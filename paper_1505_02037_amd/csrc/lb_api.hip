// lb_api.hip -- the C-ABI declared in include/lb.h (host side).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/lb.h"
#include "lb_error.h"
#include "lb_kernels.h"
#include "lb_state.h"
#include "lb_trace.h"

using lbnr::Geom;

static_assert(LB_SLICING_HARMONIC == lbnr::kSlicingHarmonic && LB_SLICING_GEODESIC == lbnr::kSlicingGeodesic &&
                  LB_SLICING_ONE_PLUS_LOG == lbnr::kSlicingOnePlusLog,
              "slicing codes of the C-ABI and the kernels");
static_assert(LB_MATTER_TENSOR == lbnr::kMatterTensor && LB_MATTER_FLUID == lbnr::kMatterFluid,
              "matter kinds of the C-ABI and the kernels");
static_assert(LB_COLLISION_BGK == lbnr::kCollisionBgk && LB_COLLISION_REGULARIZED == lbnr::kCollisionRegularized,
              "collision kinds of the C-ABI and the kernels");

namespace {
thread_local char g_last_error[256] = "";
} // namespace

void lbnr::set_last_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
}

namespace {

int fail_hip(hipError_t e, const char *what)
{
    lbnr::set_last_error("%s: %s", what, hipGetErrorString(e));
    return LB_EDEVICE;
}

#define LB_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return fail_hip(e_, #call);    \
    } while (0)

// Keeps the caller's current device and restores it on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (dev < 0 || dev == prev) || hipSetDevice(dev) == hipSuccess;
        if (!ok) (void)hipGetLastError(); // the refusal is reported by the caller, not by a later launch check
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Makes the handle's device current for the scope of a call (an error if it
// cannot be made current).
#define LB_ON_DEVICE(h)                                                  \
    DeviceGuard dg_(h->device);                                          \
    if (!dg_.ok) return fail_hip(hipErrorInvalidDevice, "hipSetDevice")

size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// padding of every (field, direction) plane, in elements (5 blocks of 64)
constexpr size_t kPlanePad = 320;

} // namespace

struct lb_handle {
    lb_config cfg;
    Geom G;
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *fbuf[2] = {nullptr, nullptr};   // distribution buffers [16][Q][ps] (double or float)
    double *ubar = nullptr;               // [16][ps] moments of the current state
    double *ubar2 = nullptr;              // [16][ps] next step's moments (fused path)
    bool ubar_valid = false;              // ubar holds the current state's moments
    bool fused = false;                   // one launch per step
    double *lm = nullptr;                 // [7][ps]
    lbnr::MatterArg matter;               // matter in the sources (kind < 0: vacuum)
    double *matter_buf = nullptr;         // [10][ps] per-site matter values, allocated on first use
    int cur = 0;                          // buffer holding the current state
    bool initialised = false;
    long long steps = 0;
    double omega = 0.0, srcfac = 0.0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    double ms_moments = 0.0, ms_collide = 0.0; // fused path: ms_moments holds the one kernel
    bool timed_fused = false;
    bool timed_matter = false;
    long long timed_launches = 0;
};

namespace {

// device memory of a handle: the caller's allocator if the config names one
hipError_t dev_malloc(lb_handle *h, void **p, size_t bytes)
{
    if (h->cfg.dev_alloc) {
        *p = h->cfg.dev_alloc(bytes, h->cfg.alloc_ctx);
        if (!*p) lbnr::set_last_error("dev_alloc returned NULL for %zu bytes", bytes);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        lbnr::set_last_error("hipMalloc: %s", hipGetErrorString(e));
        (void)hipGetLastError();
    }
    return e;
}

void dev_release(lb_handle *h, void *p)
{
    if (!p) return;
    if (h->cfg.dev_free)
        h->cfg.dev_free(p, h->cfg.alloc_ctx);
    else
        (void)hipFree(p);
}

int validate(const lb_config *c)
{
    if (!c) return LB_EINVAL;
    if ((c->dev_alloc == nullptr) != (c->dev_free == nullptr)) return LB_EINVAL;
    if (c->lattice != LB_D3Q19 && c->lattice != LB_D2Q9) return LB_EINVAL;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return LB_EINVAL;
    // D2Q9 is a lattice one site thick in z, stepped by the split launches
    if (c->lattice == LB_D2Q9 && (c->nz != 1 || c->path == LB_PATH_FUSED)) return LB_EINVAL;
    const double n = (double)c->nx * (double)c->ny * (double)c->nz;
    if (n > 4294967295.0) return LB_EINVAL; // 32-bit site indices
    if (!(c->tau > 0.5) || !isfinite(c->tau)) return LB_EINVAL;
    if (c->slicing != LB_SLICING_HARMONIC && c->slicing != LB_SLICING_GEODESIC &&
        c->slicing != LB_SLICING_ONE_PLUS_LOG)
        return LB_EINVAL;
    if (c->precision != LB_FP64 && c->precision != LB_FP32_DEV) return LB_EINVAL;
    if (c->path != LB_PATH_AUTO && c->path != LB_PATH_SPLIT && c->path != LB_PATH_FUSED) return LB_EINVAL;
    if (c->collision != LB_COLLISION_BGK && c->collision != LB_COLLISION_REGULARIZED) return LB_EINVAL;
    // the z-marching launch relaxes with BGK only
    if (c->collision != LB_COLLISION_BGK && c->path == LB_PATH_FUSED) return LB_EINVAL;
    return LB_OK;
}

Geom geom_of(const lb_config *c)
{
    Geom G;
    G.nx = c->nx;
    G.ny = c->ny;
    G.nz = c->nz;
    G.nsite = (uint32_t)((size_t)c->nx * c->ny * c->nz);
    // planes of a power-of-two size (256^3 sites: 2^27 bytes) would put a
    // site's 19 pulls and its paired stores at power-of-two strides; an odd
    // number of 64-element blocks of padding staggers them (the FP32 step at
    // 256^3 ran ~3 % faster, the FP64 step unchanged)
    G.ps = round_up(G.nsite, 64) + kPlanePad;
    G.nq = c->lattice;
    return G;
}

size_t elem_bytes(int precision) { return precision == LB_FP32_DEV ? sizeof(float) : sizeof(double); }
size_t dist_bytes(const Geom &G, int precision) { return (size_t)16 * G.nq * G.ps * elem_bytes(precision); }

// the buffer not holding the current state: free scratch between steps
// (at least 16 x 9 x 4 bytes per site: 18 doubles)
double *spare(lb_handle *h) { return (double *)h->fbuf[h->cur ^ 1]; }

bool fp32(const lb_handle *h) { return h->cfg.precision == LB_FP32_DEV; }

// moments and corrected lapse/metric of the current state
hipError_t run_moments(lb_handle *h)
{
    const int slicing = h->cfg.slicing;
    if (fp32(h))
        return lbnr::launch_moments32((const float *)h->fbuf[h->cur], h->G, slicing, h->ubar, h->lm, h->stream);
    return lbnr::launch_moments((const double *)h->fbuf[h->cur], h->G, slicing, h->ubar, h->lm, h->stream);
}

hipError_t run_collide(lb_handle *h)
{
    const int slicing = h->cfg.slicing;
    if (fp32(h))
        return lbnr::launch_collide32((const float *)h->fbuf[h->cur], (float *)h->fbuf[h->cur ^ 1], h->G, slicing,
                                      h->omega, h->srcfac, h->ubar, h->lm, h->matter, h->cfg.collision, h->stream);
    return lbnr::launch_collide((const double *)h->fbuf[h->cur], (double *)h->fbuf[h->cur ^ 1], h->G, slicing,
                                h->omega, h->srcfac, h->ubar, h->lm, h->matter, h->cfg.collision, h->stream);
}

// gives back every device buffer (the handle's stream must be idle)
void free_all(lb_handle *h)
{
    for (int i = 0; i < 2; ++i) dev_release(h, h->fbuf[i]);
    dev_release(h, h->ubar);
    dev_release(h, h->ubar2);
    dev_release(h, h->lm);
    dev_release(h, h->matter_buf);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

int ensure_events(lb_handle *h, size_t n)
{
    while (h->events.size() < n) {
        hipEvent_t e;
        LB_HIP(hipEventCreate(&e));
        h->events.push_back(e);
    }
    return LB_OK;
}

} // namespace

extern "C" {

size_t lb_device_bytes(const lb_config *cfg)
{
    if (validate(cfg) != LB_OK) return 0;
    const Geom G = geom_of(cfg);
    const size_t scratch = cfg->path == LB_PATH_FUSED ? 16 + 16 + 7 : 16 + 7;
    return 2 * dist_bytes(G, cfg->precision) + scratch * G.ps * sizeof(double);
}

int lb_create(const lb_config *cfg, lb_handle **out)
{
    if (!out) return LB_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != LB_OK) return rc;
    DeviceGuard dg(cfg->device);
    if (!dg.ok) return fail_hip(hipErrorInvalidDevice, "hipSetDevice");
    lb_handle *h = new (std::nothrow) lb_handle();
    if (!h) return LB_ENOMEM;
    h->cfg = *cfg;
    h->G = geom_of(cfg);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail_hip(hipErrorInvalidDevice, "hipGetDevice");
    }
    h->omega = 1.0 / cfg->tau;
    h->srcfac = 1.0 - 0.5 * h->omega; // (1 - dt / (2 tau))
    const Geom &G = h->G;
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = dev_malloc(h, &h->fbuf[i], dist_bytes(G, cfg->precision));
    if (e == hipSuccess) e = dev_malloc(h, (void **)&h->ubar, (size_t)16 * G.ps * sizeof(double));
    // the fused launch re-fetches the lines its 16-wide tile rows share with
    // neighbouring tiles, so the split launches are faster on large lattices:
    // AUTO selects them
    h->fused = cfg->path == LB_PATH_FUSED;
    if (e == hipSuccess && h->fused) e = dev_malloc(h, (void **)&h->ubar2, (size_t)16 * G.ps * sizeof(double));
    if (e == hipSuccess) e = dev_malloc(h, (void **)&h->lm, (size_t)7 * G.ps * sizeof(double));
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE;
    }
    if (cfg->stream) {
        h->stream = (hipStream_t)cfg->stream;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            free_all(h);
            delete h;
            return fail_hip(e, "hipStreamCreateWithFlags");
        }
        h->own_stream = true;
    }
    *out = h;
    return LB_OK;
}

void lb_destroy(lb_handle *h)
{
    if (!h) return;
    DeviceGuard dg(h->device); // best effort: the memory is released either way
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
}

int lb_init_fields(lb_handle *h, const double *u0, int on_device)
{
    lbnr::TraceRange trace("lb_init_fields");
    if (!h || !u0) return LB_EINVAL;
    LB_ON_DEVICE(h);
    const Geom &G = h->G;
    const size_t ubytes = (size_t)16 * G.nsite * sizeof(double);
    const double *du0 = u0;
    if (!on_device) {
        double *stage = spare(h);
        LB_HIP(hipMemcpyAsync(stage, u0, ubytes, hipMemcpyHostToDevice, h->stream));
        du0 = stage;
    }
    const int slicing = h->cfg.slicing;
    if (fp32(h))
        LB_HIP(lbnr::launch_init32(G, slicing, du0, h->lm, (float *)h->fbuf[h->cur], h->matter, h->stream));
    else
        LB_HIP(lbnr::launch_init(G, slicing, du0, h->lm, (double *)h->fbuf[h->cur], h->matter, h->stream));
    // the caller may release u0 as soon as this returns
    LB_HIP(hipStreamSynchronize(h->stream));
    h->initialised = true;
    h->ubar_valid = false;
    h->steps = 0;
    return LB_OK;
}

int lb_step(lb_handle *h, long long nsteps)
{
    lbnr::TraceRange trace("lb_step");
    if (!h || nsteps < 0) return LB_EINVAL;
    if (!h->initialised) return LB_ESTATE;
    if (nsteps == 0) return LB_OK;
    LB_ON_DEVICE(h);
    const int slicing = h->cfg.slicing;
    if (h->fused && !h->ubar_valid) {
        // the fused step starts from the current state's moments
        LB_HIP(run_moments(h));
        h->ubar_valid = true;
    }
    const int per_step = h->fused ? 1 : 2;
    // a timed call runs in chunks of at most kTimedChunk steps, each bracketed
    // by its own events and synchronised, so the event count stays bounded
    constexpr long long kTimedChunk = 256;
    double tm = 0.0, tc = 0.0;
    for (long long done = 0; done < nsteps;) {
        const long long n = h->timing && nsteps - done > kTimedChunk ? kTimedChunk : nsteps - done;
        if (h->timing) {
            int rc = ensure_events(h, (size_t)per_step * n + 1);
            if (rc != LB_OK) return rc;
            LB_HIP(hipEventRecord(h->events[0], h->stream));
        }
        for (long long s = 0; s < n; ++s) {
            if (h->fused) {
                if (fp32(h))
                    LB_HIP(lbnr::launch_fused32((const float *)h->fbuf[h->cur], (float *)h->fbuf[h->cur ^ 1], h->G,
                                                slicing, h->omega, h->srcfac, h->ubar, h->ubar2, h->stream));
                else
                    LB_HIP(lbnr::launch_fused64((const double *)h->fbuf[h->cur], (double *)h->fbuf[h->cur ^ 1],
                                                h->G, slicing, h->omega, h->srcfac, h->ubar, h->ubar2, h->stream));
                double *t = h->ubar;
                h->ubar = h->ubar2;
                h->ubar2 = t;
                if (h->timing) LB_HIP(hipEventRecord(h->events[s + 1], h->stream));
            } else {
                LB_HIP(run_moments(h));
                if (h->timing) LB_HIP(hipEventRecord(h->events[2 * s + 1], h->stream));
                LB_HIP(run_collide(h));
                if (h->timing) LB_HIP(hipEventRecord(h->events[2 * s + 2], h->stream));
                h->ubar_valid = false;
            }
            h->cur ^= 1;
            h->steps++;
        }
        if (h->timing) {
            LB_HIP(hipStreamSynchronize(h->stream));
            for (long long s = 0; s < n; ++s) {
                float a = 0.f, b = 0.f;
                if (h->fused) {
                    LB_HIP(hipEventElapsedTime(&a, h->events[s], h->events[s + 1]));
                } else {
                    LB_HIP(hipEventElapsedTime(&a, h->events[2 * s], h->events[2 * s + 1]));
                    LB_HIP(hipEventElapsedTime(&b, h->events[2 * s + 1], h->events[2 * s + 2]));
                }
                tm += a;
                tc += b;
            }
        }
        done += n;
    }
    if (h->timing) {
        h->ms_moments = tm / (double)nsteps;
        h->ms_collide = tc / (double)nsteps;
        h->timed_launches = nsteps;
        h->timed_fused = h->fused;
        h->timed_matter = h->matter.kind >= 0;
    }
    return LB_OK;
}

int lb_moments(lb_handle *h, double *u_out, int on_device)
{
    lbnr::TraceRange trace("lb_moments");
    if (!h || !u_out) return LB_EINVAL;
    if (!h->initialised) return LB_ESTATE;
    LB_ON_DEVICE(h);
    const Geom &G = h->G;
    const int slicing = h->cfg.slicing;
    double *dst = on_device ? u_out : spare(h);
    LB_HIP(run_moments(h));
    LB_HIP(lbnr::launch_output(G, slicing, h->ubar, h->lm, dst, h->matter, h->stream));
    if (!on_device)
        LB_HIP(hipMemcpyAsync(u_out, dst, (size_t)16 * G.nsite * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LB_HIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_get_distributions(lb_handle *h, double *f_out, int on_device)
{
    lbnr::TraceRange trace("lb_get_distributions");
    if (!h || !f_out) return LB_EINVAL;
    if (!h->initialised) return LB_ESTATE;
    LB_ON_DEVICE(h);
    const Geom &G = h->G;
    if (fp32(h)) {
        // one field at a time: the spare buffer holds Q doubles per site
        const size_t n = (size_t)G.nq * G.nsite;
        for (int F = 0; F < 16; ++F) {
            double *dst = on_device ? f_out + (size_t)F * n : spare(h);
            LB_HIP(lbnr::launch_gather32((const float *)h->fbuf[h->cur], G, F, dst, h->stream));
            if (!on_device)
                LB_HIP(hipMemcpyAsync(f_out + (size_t)F * n, dst, n * sizeof(double), hipMemcpyDeviceToHost,
                                      h->stream));
            if (!on_device) LB_HIP(hipStreamSynchronize(h->stream));
        }
        LB_HIP(hipStreamSynchronize(h->stream));
        return LB_OK;
    }
    double *dst = on_device ? f_out : spare(h);
    LB_HIP(lbnr::launch_gather((const double *)h->fbuf[h->cur], G, dst, h->stream));
    if (!on_device)
        LB_HIP(hipMemcpyAsync(f_out, dst, (size_t)16 * G.nq * G.nsite * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    LB_HIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_set_distributions(lb_handle *h, const double *f_in, int on_device)
{
    lbnr::TraceRange trace("lb_set_distributions");
    if (!h || !f_in) return LB_EINVAL;
    LB_ON_DEVICE(h);
    const Geom &G = h->G;
    const size_t n = (size_t)G.nq * G.nsite; // doubles per field
    if (fp32(h)) {
        // one field at a time through the spare buffer (Q doubles per site)
        for (int F = 0; F < 16; ++F) {
            const double *src = f_in + (size_t)F * n;
            if (!on_device) {
                double *stage = spare(h);
                LB_HIP(hipMemcpyAsync(stage, src, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
                src = stage;
            }
            LB_HIP(lbnr::launch_scatter32(src, G, F, (float *)h->fbuf[h->cur], h->stream));
            if (!on_device) LB_HIP(hipStreamSynchronize(h->stream));
        }
    } else {
        const double *src = f_in;
        if (!on_device) {
            double *stage = spare(h);
            LB_HIP(hipMemcpyAsync(stage, f_in, 16 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
            src = stage;
        }
        LB_HIP(lbnr::launch_scatter(src, G, (double *)h->fbuf[h->cur], h->stream));
    }
    LB_HIP(hipStreamSynchronize(h->stream));
    h->initialised = true;
    h->ubar_valid = false;
    h->steps = 0;
    return LB_OK;
}

int lb_check_finite(lb_handle *h, int *all_finite)
{
    lbnr::TraceRange trace("lb_check_finite");
    if (!h || !all_finite) return LB_EINVAL;
    if (!h->initialised) return LB_ESTATE;
    LB_ON_DEVICE(h);
    int *scratch = (int *)spare(h);
    LB_HIP(run_moments(h));
    LB_HIP(lbnr::launch_finite(h->G, h->ubar, scratch, h->stream));
    int bad = 1;
    LB_HIP(hipMemcpyAsync(&bad, scratch + lbnr::finite_scratch_ints(h->G) - 1, sizeof(int), hipMemcpyDeviceToHost,
                          h->stream));
    LB_HIP(hipStreamSynchronize(h->stream));
    *all_finite = bad ? 0 : 1;
    return LB_OK;
}

int lb_error_norms(lb_handle *h, const double *u_ref, int on_device, double *max_abs, double *l2, double *ref_max)
{
    lbnr::TraceRange trace("lb_error_norms");
    if (!h || !u_ref) return LB_EINVAL;
    if (!h->initialised) return LB_ESTATE;
    LB_ON_DEVICE(h);
    const Geom &G = h->G;
    const int slicing = h->cfg.slicing;
    // spare buffer layout: [u 16 x nsite][ref 16 x nsite][norm scratch]
    double *u = spare(h);
    double *ref = u + (size_t)16 * G.nsite;
    double *scratch = ref + (size_t)16 * G.nsite;
    LB_HIP(run_moments(h));
    LB_HIP(lbnr::launch_output(G, slicing, h->ubar, h->lm, u, h->matter, h->stream));
    const double *dref = u_ref;
    if (!on_device) {
        LB_HIP(hipMemcpyAsync(ref, u_ref, (size_t)16 * G.nsite * sizeof(double), hipMemcpyHostToDevice, h->stream));
        dref = ref;
    }
    LB_HIP(lbnr::launch_norms(G, u, dref, scratch, h->stream));
    const size_t nb = (G.nsite + 255) / 256;
    double res[16 * 3];
    LB_HIP(hipMemcpyAsync(res, scratch + nb * 16 * 3, sizeof res, hipMemcpyDeviceToHost, h->stream));
    LB_HIP(hipStreamSynchronize(h->stream));
    for (int F = 0; F < 16; ++F) {
        if (max_abs) max_abs[F] = res[F * 3 + 0];
        if (l2) l2[F] = res[F * 3 + 1];
        if (ref_max) ref_max[F] = res[F * 3 + 2];
    }
    return LB_OK;
}

int lb_set_matter(lb_handle *h, int kind, const double *M, int per_site, int on_device)
{
    if (!h) return LB_EINVAL;
    if (kind != LB_MATTER_TENSOR && kind != LB_MATTER_FLUID) return LB_EINVAL;
    if (!M) {
        h->matter.kind = -1;
        h->matter.field = nullptr;
        return LB_OK;
    }
    if (h->fused) return LB_EINVAL; // the z-marching launch evaluates vacuum sources only
    LB_ON_DEVICE(h);
    const int nc = kind == LB_MATTER_FLUID ? 2 : 10;
    const Geom &G = h->G;
    if (!per_site) {
        double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (on_device) {
            LB_HIP(hipMemcpyAsync(v, M, nc * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            LB_HIP(hipStreamSynchronize(h->stream));
        } else {
            for (int c = 0; c < nc; ++c) v[c] = M[c];
        }
        // carried by value in the arguments of every later launch
        for (int c = 0; c < 10; ++c) h->matter.uni[c] = v[c];
        h->matter.field = nullptr;
        h->matter.kind = kind;
        return LB_OK;
    }
    if (!h->matter_buf) {
        hipError_t e = dev_malloc(h, (void **)&h->matter_buf, (size_t)10 * G.ps * sizeof(double));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE;
    }
    // [nc][nsite] into planes of ps; ordered after the launches already queued
    LB_HIP(hipMemcpy2DAsync(h->matter_buf, G.ps * sizeof(double), M, (size_t)G.nsite * sizeof(double),
                            (size_t)G.nsite * sizeof(double), nc,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    if (!on_device) LB_HIP(hipStreamSynchronize(h->stream));
    h->matter.field = h->matter_buf;
    h->matter.kind = kind;
    return LB_OK;
}

long long lb_steps_done(const lb_handle *h) { return h ? h->steps : -1; }

int lb_set_timing(lb_handle *h, int enable)
{
    if (!h) return LB_EINVAL;
    h->timing = enable != 0;
    return LB_OK;
}

int lb_kernel_times(lb_handle *h, const char **names, double *ms, int cap, int *count)
{
    if (!h || !count) return LB_EINVAL;
    if (h->timed_launches == 0) return LB_ESTATE;
    // the kernels' own (template instance) names, as a profiler lists them
    static const char *kMom[2][2] = {{"lbnr::k_moments<lbnr::D3Q19>", "lbnr::k_moments<lbnr::D2Q9>"},
                                     {"lbnr::k_moments32<lbnr::D3Q19>", "lbnr::k_moments32<lbnr::D2Q9>"}};
    static const char *kCol[2][2][2][2] = {
        {{{"lbnr::k_collide<lbnr::D3Q19, false, 0>", "lbnr::k_collide<lbnr::D3Q19, false, 1>"},
          {"lbnr::k_collide<lbnr::D3Q19, true, 0>", "lbnr::k_collide<lbnr::D3Q19, true, 1>"}},
         {{"lbnr::k_collide<lbnr::D2Q9, false, 0>", "lbnr::k_collide<lbnr::D2Q9, false, 1>"},
          {"lbnr::k_collide<lbnr::D2Q9, true, 0>", "lbnr::k_collide<lbnr::D2Q9, true, 1>"}}},
        {{{"lbnr::k_collide32<lbnr::D3Q19, false, 0>", "lbnr::k_collide32<lbnr::D3Q19, false, 1>"},
          {"lbnr::k_collide32<lbnr::D3Q19, true, 0>", "lbnr::k_collide32<lbnr::D3Q19, true, 1>"}},
         {{"lbnr::k_collide32<lbnr::D2Q9, false, 0>", "lbnr::k_collide32<lbnr::D2Q9, false, 1>"},
          {"lbnr::k_collide32<lbnr::D2Q9, true, 0>", "lbnr::k_collide32<lbnr::D2Q9, true, 1>"}}}};
    static const char *kFused[2] = {"lbnr::k_fused<double>", "lbnr::k_fused<float>"};
    const int f32 = fp32(h) ? 1 : 0, q9 = h->G.nq == LB_D2Q9 ? 1 : 0, mat = h->timed_matter ? 1 : 0;
    const int coll = h->cfg.collision == LB_COLLISION_REGULARIZED ? 1 : 0;
    const char *kNames[2] = {h->timed_fused ? kFused[f32] : kMom[f32][q9], kCol[f32][q9][mat][coll]};
    const int nk = h->timed_fused ? 1 : 2;
    const double vals[2] = {h->ms_moments, h->ms_collide};
    int n = 0;
    for (int i = 0; i < nk && i < cap; ++i, ++n) {
        if (names) names[i] = kNames[i];
        if (ms) ms[i] = vals[i];
    }
    *count = n;
    return LB_OK;
}

const char *lb_strerror(int code)
{
    switch (code) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "out of device memory";
    case LB_EDEVICE: return "HIP runtime error";
    case LB_ESTATE: return "handle not initialised";
    default: return "unknown error";
    }
}

const char *lb_last_error(void) { return g_last_error; }

} // extern "C"
