// lb_serve.hip -- continuous batching of independent evolutions (include/lb_serve.h).
//
// Device side: every resident request has a descriptor (lattice geometry,
// relaxation parameters, buffer pointers, current-buffer parity and steps
// remaining).  A work list enumerates (request, 256-site block) items of all
// resident requests; the batched kernels stride over it with a grid sized to
// the machine and run the same per-site step as the single-lattice kernels.
// A bookkeeping kernel flips each active request's parity and counts its step
// down, so a captured graph of K steps stops every request at its own count.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <map>
#include <new>
#include <vector>

#include "../../include/lb.h"
#include "../../include/lb_serve.h"
#include "lb_error.h"
#include "lb_kernels.h"
#include "lb_site.h"
#include "lb_step.h"
#include "lb_trace.h"

namespace lbnr {

struct ReqDesc {
    Geom G;
    double omega, srcfac;
    int slicing;
    int cur;              // buffer holding the current state (device-updated)
    long long remaining;  // steps left (device-updated)
    void *f[2];
    double *ubar;
    double *lm;
};

struct WorkItem {
    int req;
    uint32_t first; // first site of the 256-site block
};

template <bool kF32>
__global__ void __launch_bounds__(256) k_serve_moments(const ReqDesc *__restrict__ R, const WorkItem *__restrict__ W,
                                                       int nitems)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const WorkItem w = W[it];
        const ReqDesc &r = R[w.req];
        if (r.remaining <= 0) continue;
        const uint32_t s = w.first + threadIdx.x;
        if (s >= r.G.nsite) continue;
        if constexpr (kF32)
            moments_site32((const float *)r.f[r.cur], r.G, s, r.slicing, r.ubar, r.lm);
        else
            moments_site64((const double *)r.f[r.cur], r.G, s, r.slicing, r.ubar, r.lm);
    }
}

template <bool kF32>
__global__ void __launch_bounds__(256) k_serve_collide(const ReqDesc *__restrict__ R, const WorkItem *__restrict__ W,
                                                       int nitems)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const WorkItem w = W[it];
        const ReqDesc &r = R[w.req];
        if (r.remaining <= 0) continue;
        const uint32_t s = w.first + threadIdx.x;
        if (s >= r.G.nsite) continue;
        if constexpr (kF32)
            collide_site32((const float *)r.f[r.cur], (float *)r.f[r.cur ^ 1], r.G, s, r.slicing, r.omega,
                           r.srcfac, r.ubar, r.lm);
        else
            collide_site64((const double *)r.f[r.cur], (double *)r.f[r.cur ^ 1], r.G, s, r.slicing, r.omega,
                           r.srcfac, r.ubar, r.lm);
    }
}

__global__ void k_serve_advance(ReqDesc *__restrict__ R, int nreq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nreq && R[i].remaining > 0) {
        R[i].cur ^= 1;
        R[i].remaining -= 1;
    }
}

} // namespace lbnr

using lbnr::Geom;
using lbnr::ReqDesc;
using lbnr::WorkItem;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int hip_fail(hipError_t e, const char *what)
{
    lbnr::set_last_error("%s: %s", what, hipGetErrorString(e));
    fprintf(stderr, "lb_serve: %s: %s\n", what, hipGetErrorString(e));
    return LB_EDEVICE;
}

#define SV_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

// Keeps the caller's current device and restores it on scope exit; `ok` tells
// whether the requested device could be made current.
struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (dev < 0 || dev == prev) || hipSetDevice(dev) == hipSuccess;
        if (!ok) (void)hipGetLastError(); // the refusal is reported by the caller, not by a later launch check
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

constexpr size_t kAlign = 4096;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Geom geom(const lb_config *c)
{
    Geom G;
    G.nx = c->nx;
    G.ny = c->ny;
    G.nz = c->nz;
    G.nsite = (uint32_t)((size_t)c->nx * c->ny * c->nz);
    G.ps = align_up(G.nsite, 64);
    return G;
}

// arena layout of one request: f[0], f[1], ubar[16], lm[7]
struct Layout {
    size_t f0, f1, ubar, lm, total;
};
Layout layout(const Geom &G, int precision)
{
    const size_t eb = precision == LB_FP32_DEV ? 4 : 8;
    Layout L;
    const size_t fb = align_up((size_t)16 * 19 * G.ps * eb, kAlign);
    L.f0 = 0;
    L.f1 = fb;
    L.ubar = 2 * fb;
    L.lm = L.ubar + align_up((size_t)16 * G.ps * 8, kAlign);
    L.total = L.lm + align_up((size_t)7 * G.ps * 8, kAlign);
    return L;
}

bool valid_request(const lb_config *c)
{
    if (!c || c->lattice != LB_D3Q19 || c->collision != LB_COLLISION_BGK) return false;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return false;
    if ((double)c->nx * c->ny * c->nz > 4294967295.0) return false;
    if (!(c->tau > 0.5) || !isfinite(c->tau)) return false;
    return c->slicing == LB_SLICING_HARMONIC || c->slicing == LB_SLICING_GEODESIC ||
           c->slicing == LB_SLICING_ONE_PLUS_LOG;
}

// first-fit allocator over [0, size) with coalescing
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free; // offset -> length
    size_t in_use = 0, peak = 0;
    void reset(size_t n)
    {
        size = n;
        free.clear();
        free[0] = n;
        in_use = peak = 0;
    }
    bool alloc(size_t n, size_t *off)
    {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o = it->first;
                free.erase(it);
                if (rest) free[o + n] = rest;
                in_use += n;
                if (in_use > peak) peak = in_use;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        in_use -= n;
        auto it = free.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Req {
    unsigned long long id = 0;
    lb_config cfg{};
    Geom G{};
    long long nsteps = 0;
    long long done_steps = 0;
    std::vector<double> u0;
    std::vector<double> result;
    int state = LB_REQ_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t off = 0, bytes = 0;
    Layout L{};
};

} // namespace

struct lb_server {
    lb_server_config cfg{};
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *arena_base = nullptr;
    Arena arena;
    std::map<unsigned long long, Req> reqs;
    std::vector<unsigned long long> queue;    // arrival order
    std::vector<unsigned long long> resident; // slot order
    std::vector<ReqDesc> hdesc;
    ReqDesc *ddesc = nullptr;
    WorkItem *ditems = nullptr;
    size_t items_cap = 0;
    int nitems = 0;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    unsigned long long next_id = 1;
    int ncu = 256;
    long long launches = 0, site_updates = 0, completed = 0, failed = 0;
};

namespace {

int rebuild(lb_server *s)
{
    // descriptors of the resident set (hdesc already carries device-updated
    // parity / remaining of requests that stay)
    const int nres = (int)s->resident.size();
    std::vector<WorkItem> items;
    for (int slot = 0; slot < nres; ++slot) {
        const Req &r = s->reqs[s->resident[slot]];
        for (uint32_t b = 0; b < r.G.nsite; b += 256) items.push_back({slot, b});
    }
    s->nitems = (int)items.size();
    if (nres) SV_HIP(hipMemcpyAsync(s->ddesc, s->hdesc.data(), nres * sizeof(ReqDesc), hipMemcpyHostToDevice, s->stream));
    if (items.size() > s->items_cap) {
        // the old list is dropped before the new one is allocated, so that a
        // failed allocation leaves no stale pointer for lb_server_destroy
        WorkItem *old = s->ditems;
        s->ditems = nullptr;
        s->items_cap = 0;
        if (old) SV_HIP(hipFree(old));
        SV_HIP(hipMalloc((void **)&s->ditems, items.size() * 2 * sizeof(WorkItem)));
        s->items_cap = items.size() * 2;
    }
    if (!items.empty())
        SV_HIP(hipMemcpyAsync(s->ditems, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                              s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    if (s->exec) {
        SV_HIP(hipGraphExecDestroy(s->exec));
        s->exec = nullptr;
    }
    if (nres == 0) {
        s->dirty = false;
        return LB_OK;
    }
    const bool f32 = s->cfg.precision == LB_FP32_DEV;
    const int grid = s->nitems < s->ncu * 4 ? s->nitems : s->ncu * 4;
    hipGraph_t graph = nullptr;
    SV_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < s->cfg.steps_per_launch; ++k) {
        if (f32) {
            hipLaunchKernelGGL(lbnr::k_serve_moments<true>, dim3(grid), dim3(256), 0, s->stream, s->ddesc, s->ditems,
                               s->nitems);
            hipLaunchKernelGGL(lbnr::k_serve_collide<true>, dim3(grid), dim3(256), 0, s->stream, s->ddesc, s->ditems,
                               s->nitems);
        } else {
            hipLaunchKernelGGL(lbnr::k_serve_moments<false>, dim3(grid), dim3(256), 0, s->stream, s->ddesc,
                               s->ditems, s->nitems);
            hipLaunchKernelGGL(lbnr::k_serve_collide<false>, dim3(grid), dim3(256), 0, s->stream, s->ddesc,
                               s->ditems, s->nitems);
        }
        hipLaunchKernelGGL(lbnr::k_serve_advance, dim3((nres + 63) / 64), dim3(64), 0, s->stream, s->ddesc, nres);
    }
    hipError_t e = hipStreamEndCapture(s->stream, &graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    s->dirty = false;
    return LB_OK;
}

int admit(lb_server *s)
{
    const bool f32 = s->cfg.precision == LB_FP32_DEV;
    std::vector<unsigned long long> still;
    for (unsigned long long id : s->queue) {
        Req &r = s->reqs[id];
        size_t off = 0;
        if ((int)s->resident.size() >= s->cfg.max_resident || !s->arena.alloc(r.L.total, &off)) {
            still.push_back(id);
            continue;
        }
        r.off = off;
        r.bytes = r.L.total;
        char *base = s->arena_base + off;
        ReqDesc d{};
        d.G = r.G;
        d.omega = 1.0 / r.cfg.tau;
        d.srcfac = 1.0 - 0.5 * d.omega;
        d.slicing = r.cfg.slicing;
        d.cur = 0;
        d.remaining = r.nsteps;
        d.f[0] = base + r.L.f0;
        d.f[1] = base + r.L.f1;
        d.ubar = (double *)(base + r.L.ubar);
        d.lm = (double *)(base + r.L.lm);
        // initial distributions, u0 staged in the second buffer
        double *stage = (double *)d.f[1];
        SV_HIP(hipMemcpyAsync(stage, r.u0.data(), r.u0.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
        if (f32)
            SV_HIP(lbnr::launch_init32(r.G, d.slicing, stage, d.lm, (float *)d.f[0], lbnr::MatterArg{}, s->stream));
        else
            SV_HIP(lbnr::launch_init(r.G, d.slicing, stage, d.lm, (double *)d.f[0], lbnr::MatterArg{}, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        std::vector<double>().swap(r.u0);
        r.state = LB_REQ_RUNNING;
        r.t_admit = now_s();
        s->resident.push_back(id);
        s->hdesc.push_back(d);
        s->dirty = true;
    }
    s->queue.swap(still);
    return LB_OK;
}

int harvest(lb_server *s)
{
    const int nres = (int)s->resident.size();
    if (!nres) return LB_OK;
    std::vector<ReqDesc> now(nres);
    SV_HIP(hipMemcpyAsync(now.data(), s->ddesc, nres * sizeof(ReqDesc), hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    const bool f32 = s->cfg.precision == LB_FP32_DEV;
    std::vector<unsigned long long> keep;
    std::vector<ReqDesc> keepd;
    for (int slot = 0; slot < nres; ++slot) {
        Req &r = s->reqs[s->resident[slot]];
        const ReqDesc &d = now[slot];
        s->site_updates += (long long)(s->hdesc[slot].remaining - d.remaining) * (long long)r.G.nsite;
        r.done_steps = r.nsteps - d.remaining;
        if (d.remaining > 0) {
            keep.push_back(r.id);
            keepd.push_back(d);
            continue;
        }
        // finished: u = ubar + R/2 into the spare buffer, then to the host
        double *out = (double *)d.f[d.cur ^ 1];
        if (f32)
            SV_HIP(lbnr::launch_moments32((const float *)d.f[d.cur], r.G, d.slicing, d.ubar, d.lm, s->stream));
        else
            SV_HIP(lbnr::launch_moments((const double *)d.f[d.cur], r.G, d.slicing, d.ubar, d.lm, s->stream));
        SV_HIP(lbnr::launch_output(r.G, d.slicing, d.ubar, d.lm, out, lbnr::MatterArg{}, s->stream));
        r.result.resize((size_t)16 * r.G.nsite);
        SV_HIP(hipMemcpyAsync(r.result.data(), out, r.result.size() * sizeof(double), hipMemcpyDeviceToHost,
                              s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        bool finite = true;
        for (double v : r.result)
            if (!isfinite(v)) {
                finite = false;
                break;
            }
        r.state = finite ? LB_REQ_DONE : LB_REQ_FAILED;
        (finite ? s->completed : s->failed)++;
        r.t_done = now_s();
        s->arena.release(r.off, r.bytes);
        s->dirty = true;
    }
    s->resident.swap(keep);
    s->hdesc.swap(keepd);
    return LB_OK;
}

} // namespace

extern "C" {

int lb_server_create(const lb_server_config *cfg, lb_server **out)
{
    if (!out) return LB_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget_bytes < kAlign || cfg->max_resident < 1 || cfg->steps_per_launch < 1)
        return LB_EINVAL;
    if (cfg->precision != LB_FP64 && cfg->precision != LB_FP32_DEV) return LB_EINVAL;
    DevGuard dg(cfg->device);
    if (!dg.ok) return hip_fail(hipErrorInvalidDevice, "hipSetDevice");
    lb_server *s = new (std::nothrow) lb_server();
    if (!s) return LB_ENOMEM;
    s->cfg = *cfg;
    s->cfg.hbm_budget_bytes = cfg->hbm_budget_bytes / kAlign * kAlign;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return LB_EDEVICE;
    }
    (void)hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->device);
    hipError_t e = hipMalloc((void **)&s->arena_base, s->cfg.hbm_budget_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&s->ddesc, (size_t)cfg->max_resident * sizeof(ReqDesc));
    if (e == hipSuccess) {
        if (cfg->stream) {
            s->stream = (hipStream_t)cfg->stream;
        } else {
            e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            s->own_stream = e == hipSuccess;
        }
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (s->arena_base) (void)hipFree(s->arena_base);
        if (s->ddesc) (void)hipFree(s->ddesc);
        delete s;
        lbnr::set_last_error("lb_server_create: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE;
    }
    s->arena.reset(s->cfg.hbm_budget_bytes);
    *out = s;
    return LB_OK;
}

size_t lb_server_request_bytes(const lb_server *s, const lb_config *cfg)
{
    if (!s || !valid_request(cfg)) return 0;
    return layout(geom(cfg), s->cfg.precision).total;
}

int lb_server_submit(lb_server *s, const lb_config *cfg, const double *u0, long long nsteps, unsigned long long *id)
{
    if (!s || !u0 || !id || nsteps < 0 || !valid_request(cfg)) return LB_EINVAL;
    Req r;
    r.id = s->next_id++;
    r.cfg = *cfg;
    r.G = geom(cfg);
    r.L = layout(r.G, s->cfg.precision);
    if (r.L.total > s->arena.size) return LB_EINVAL;
    r.nsteps = nsteps;
    r.u0.assign(u0, u0 + (size_t)16 * r.G.nsite);
    r.t_submit = now_s();
    *id = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    return LB_OK;
}

int lb_server_advance(lb_server *s, int *active)
{
    lbnr::TraceRange trace("lb_server_advance");
    if (!s) return LB_EINVAL;
    DevGuard dg(s->device);
    if (!dg.ok) return hip_fail(hipErrorInvalidDevice, "hipSetDevice");
    int rc = admit(s);
    if (rc != LB_OK) return rc;
    if (s->dirty) {
        rc = rebuild(s);
        if (rc != LB_OK) return rc;
    }
    if (!s->resident.empty()) {
        SV_HIP(hipGraphLaunch(s->exec, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        s->launches++;
        rc = harvest(s);
        if (rc != LB_OK) return rc;
        if (s->dirty) {
            // keep the graph in step with the resident set for the next round
            rc = admit(s);
            if (rc == LB_OK) rc = rebuild(s);
            if (rc != LB_OK) return rc;
        }
    }
    if (active) *active = (int)(s->resident.size() + s->queue.size());
    return LB_OK;
}

int lb_server_info(const lb_server *s, unsigned long long id, lb_request_info *info)
{
    if (!s || !info) return LB_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return LB_EINVAL;
    const Req &r = it->second;
    info->state = r.state;
    info->steps_done = r.done_steps;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_done = r.t_done;
    return LB_OK;
}

int lb_server_result(lb_server *s, unsigned long long id, double *u_out)
{
    if (!s || !u_out) return LB_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return LB_EINVAL;
    Req &r = it->second;
    if (r.state != LB_REQ_DONE && r.state != LB_REQ_FAILED) return LB_ESTATE;
    memcpy(u_out, r.result.data(), r.result.size() * sizeof(double));
    s->reqs.erase(it);
    return LB_OK;
}

int lb_server_get_stats(const lb_server *s, lb_server_stats *st)
{
    if (!s || !st) return LB_EINVAL;
    st->graph_launches = s->launches;
    st->site_updates = s->site_updates;
    st->completed = s->completed;
    st->failed = s->failed;
    st->resident = (int)s->resident.size();
    st->queued = (int)s->queue.size();
    st->arena_bytes = s->arena.size;
    st->arena_in_use = s->arena.in_use;
    st->arena_peak = s->arena.peak;
    return LB_OK;
}

void lb_server_destroy(lb_server *s)
{
    if (!s) return;
    DevGuard dg(s->device); // best effort: the memory is released either way
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->ditems) (void)hipFree(s->ditems);
    if (s->ddesc) (void)hipFree(s->ddesc);
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

} // extern "C"
