// lb_fp64.hip -- FP64 kernels of the Bona-Masso lattice Boltzmann step.
//
// Storage (pull scheme).  A distribution buffer holds the post-collision
// values f*_{F,q}(x) of the previous step, SoA [field][q][plane] (q over the
// 19 directions of D3Q19 or the 9 of D2Q9), one plane of
// `ps` doubles per (field, direction) with x fastest (ps = nsite rounded up to
// 64 elements, so every plane starts 512-byte aligned).  The distribution at
// the current time is f_{F,q}(x) = buf[F][q][x - c_q] (periodic wrap).
//
// One time step is two launches:
//   k_moments  pulls all 16 fields at a site, sums the moments, applies the
//              local half-source correction of lapse and metric and writes
//              ubar[16] and the corrected lapse/metric lm[7] per site;
//   k_collide  reads ubar and lm at the site and lm at the six face
//              neighbours (A_k, D_kij by central differences), evaluates S_ij,
//              Omega_k and the flux, then pulls every distribution again,
//              relaxes it towards its equilibrium with the source added and
//              stores it at x in the other buffer.
#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"
#include "lb_step.h"

namespace lbnr {

// ---------------------------------------------------------------------------
// k_moments: zeroth moments of all fields and the corrected lapse/metric
// ---------------------------------------------------------------------------
template <class L>
__global__ void __launch_bounds__(256) k_moments(const double *__restrict__ fin, Geom G, int slicing,
                                                 double *__restrict__ ubar, double *__restrict__ lm)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < G.nsite) moments_site64<L>(fin, G, s, slicing, ubar, lm);
}

// ---------------------------------------------------------------------------
// k_collide: sources, flux, BGK relaxation with source, pull streaming
// ---------------------------------------------------------------------------
template <class L, bool HasMatter, int Coll>
__global__ void __launch_bounds__(256) k_collide(const double *__restrict__ fin, double *__restrict__ fout,
                                                 Geom G, int slicing, double omega, double srcfac,
                                                 const double *__restrict__ ubar, const double *__restrict__ lm,
                                                 MatterArg m)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < G.nsite) collide_site64<L, HasMatter, Coll>(fin, fout, G, s, slicing, omega, srcfac, ubar, lm, m);
}

// ---------------------------------------------------------------------------
// k_output: the half-source moments u = ubar + R/2 into an unpadded array
// ---------------------------------------------------------------------------
template <bool HasMatter>
__global__ void __launch_bounds__(256) k_output(Geom G, int slicing, const double *__restrict__ ubar,
                                                const double *__restrict__ lm, double *__restrict__ u, MatterArg m)
{
    Site o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) ub[F] = ubar[(size_t)F * G.ps + o.s];
    Params P;
    site_params<HasMatter>(G, o, slicing, ub, lm, P, m);
#pragma unroll
    for (int F = 0; F < kFields; ++F) u[(size_t)F * G.nsite + o.s] = P.u[F];
}

// ---------------------------------------------------------------------------
// initialisation from fields u0 (unpadded): f = f^eq(u0) - w R(u0)/2, every
// quantity at u0, stored where the first pull of each direction reads it
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init_lm(Geom G, const double *__restrict__ u0, double *__restrict__ lm)
{
    Site o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
#pragma unroll
    for (int F = 0; F < 7; ++F) lm[(size_t)F * G.ps + o.s] = u0[(size_t)F * G.nsite + o.s];
}

// f_q = f^eq_q - w_q R/2 for one field, direction q fixed at compile time;
// the pull of direction q at x reads position x - c_q
template <class L, int Fld, int q = 0>
__device__ __forceinline__ void init_field_q(double *__restrict__ fout, const Geom &G, const SiteT<L> &o,
                                             const Params &P, double hR)
{
    plane<L>(fout, G, Fld, q)[o.src[q]] = feq64<L, Fld, q>(P) - L::w(q) * hR;
    if constexpr (q + 1 < L::Q) init_field_q<L, Fld, q + 1>(fout, G, o, P, hR);
}

template <int Fld, class L>
__device__ __forceinline__ void init_field(double *__restrict__ fout, const Geom &G, const SiteT<L> &o,
                                           const Params &P)
{
    init_field_q<L, Fld>(fout, G, o, P, 0.5 * P.R[Fld]);
    if constexpr (Fld + 1 < kFields) init_field<Fld + 1>(fout, G, o, P);
}

template <class L, bool HasMatter>
__global__ void __launch_bounds__(256) k_init(Geom G, int slicing, const double *__restrict__ u0,
                                              const double *__restrict__ lm, double *__restrict__ fout, MatterArg m)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    double u[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) u[F] = u0[(size_t)F * G.nsite + o.s];
    Params P;
    // R_alpha, R_gamma at u0 (the corrected values are not used: u stays u0)
    double c[7], Rag[7];
    lapse_metric(u, slicing, c, Rag);
    double A[3], D[18], gi[6], S[6], Om[3];
    stencil(G, o, lm, u[0], A, D);
    sym_inverse(u + 1, gi);
    bm_sources(u[0], u + 1, gi, u + 7, u + 13, A, D, S, Om);
    if constexpr (HasMatter) {
        double M[10];
        matter_load(m, G, o.s, M);
        matter_sources(u[0], u + 1, gi, m.kind, M, S, Om);
    }
#pragma unroll
    for (int F = 0; F < kFields; ++F) P.u[F] = u[F];
#pragma unroll
    for (int F = 0; F < 7; ++F) P.R[F] = Rag[F];
#pragma unroll
    for (int p = 0; p < 6; ++p) P.R[7 + p] = u[0] * S[p];
#pragma unroll
    for (int k = 0; k < 3; ++k) P.R[13 + k] = Om[k];
    bm_flux(u[0], u + 1, gi, u + 13, A, D, P.F);
    // the stored position of direction q is x - c_q
    pull_sources(G, o);
    init_field<0>(fout, G, o, P);
}

// distributions at the current time (after streaming), unpadded
template <class L>
__global__ void __launch_bounds__(256) k_gather(const double *__restrict__ fin, Geom G, double *__restrict__ f)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    pull_sources(G, o);
#pragma unroll
    for (int F = 0; F < kFields; ++F)
#pragma unroll
        for (int q = 0; q < L::Q; ++q)
            f[((size_t)F * L::Q + q) * G.nsite + o.s] = plane<L>(fin, G, F, q)[o.src[q]];
}

// ---------------------------------------------------------------------------
// error norms: per-block partials, then one block folds them in block order
// ---------------------------------------------------------------------------
constexpr int kNormThreads = 256;

__global__ void __launch_bounds__(kNormThreads) k_norm_partial(Geom G, const double *__restrict__ u,
                                                               const double *__restrict__ ref,
                                                               double *__restrict__ part)
{
    // part[(blockIdx.x * 16 + F) * 3 + {0: max|d|, 1: sum d^2, 2: max|ref|}]
    __shared__ double smax[kNormThreads], ssum[kNormThreads], sref[kNormThreads];
    const uint32_t s = blockIdx.x * kNormThreads + threadIdx.x;
    for (int F = 0; F < kFields; ++F) {
        double dmax = 0.0, d2 = 0.0, rmax = 0.0;
        if (s < G.nsite) {
            const double r = ref[(size_t)F * G.nsite + s];
            const double d = u[(size_t)F * G.nsite + s] - r;
            dmax = fabs(d);
            d2 = d * d;
            rmax = fabs(r);
            if (d != d) dmax = d; // keep NaN visible
        }
        smax[threadIdx.x] = dmax;
        ssum[threadIdx.x] = d2;
        sref[threadIdx.x] = rmax;
        __syncthreads();
        for (int w = kNormThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const double a = smax[threadIdx.x], b = smax[threadIdx.x + w];
                smax[threadIdx.x] = (a != a || b != b) ? (a + b) : fmax(a, b);
                ssum[threadIdx.x] += ssum[threadIdx.x + w];
                sref[threadIdx.x] = fmax(sref[threadIdx.x], sref[threadIdx.x + w]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *p = part + ((size_t)blockIdx.x * kFields + F) * 3;
            p[0] = smax[0];
            p[1] = ssum[0];
            p[2] = sref[0];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kFields) k_norm_final(const double *__restrict__ part, uint32_t nblocks,
                                                        uint32_t nsite, double *__restrict__ out)
{
    const int F = threadIdx.x;
    double dmax = 0.0, d2 = 0.0, rmax = 0.0;
    for (uint32_t b = 0; b < nblocks; ++b) {
        const double *p = part + ((size_t)b * kFields + F) * 3;
        dmax = (dmax != dmax || p[0] != p[0]) ? (dmax + p[0]) : fmax(dmax, p[0]);
        d2 += p[1];
        rmax = fmax(rmax, p[2]);
    }
    out[F * 3 + 0] = dmax;
    out[F * 3 + 1] = sqrt(d2 / (double)nsite);
    out[F * 3 + 2] = rmax;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 grid_for(uint32_t n, int threads) { return dim3((n + threads - 1) / threads); }

hipError_t launch_moments(const double *fin, const Geom &G, int slicing, double *ubar, double *lm, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_moments<D2Q9>, grid_for(G.nsite, 256), dim3(256), 0, st, fin, G, slicing, ubar, lm);
    else
        hipLaunchKernelGGL(k_moments<D3Q19>, grid_for(G.nsite, 256), dim3(256), 0, st, fin, G, slicing, ubar, lm);
    return hipGetLastError();
}

template <class L, bool HasMatter>
static void collide_instance(int collision, dim3 grid, hipStream_t st, const double *fin, double *fout,
                             const Geom &G, int slicing, double omega, double srcfac, const double *ubar,
                             const double *lm, const MatterArg &m)
{
    if (collision == kCollisionRegularized)
        hipLaunchKernelGGL((k_collide<L, HasMatter, kCollisionRegularized>), grid, dim3(256), 0, st, fin, fout, G,
                           slicing, omega, srcfac, ubar, lm, m);
    else
        hipLaunchKernelGGL((k_collide<L, HasMatter, kCollisionBgk>), grid, dim3(256), 0, st, fin, fout, G, slicing,
                           omega, srcfac, ubar, lm, m);
}

hipError_t launch_collide(const double *fin, double *fout, const Geom &G, int slicing, double omega,
                          double srcfac, const double *ubar, const double *lm, const MatterArg &m, int collision,
                          hipStream_t st)
{
    const dim3 grid = grid_for(G.nsite, 256);
    const bool q9 = G.nq == D2Q9::Q, mat = m.kind >= 0;
    if (q9 && mat)
        collide_instance<D2Q9, true>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else if (q9)
        collide_instance<D2Q9, false>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else if (mat)
        collide_instance<D3Q19, true>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else
        collide_instance<D3Q19, false>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    return hipGetLastError();
}

hipError_t launch_output(const Geom &G, int slicing, const double *ubar, const double *lm, double *u,
                         const MatterArg &m, hipStream_t st)
{
    if (m.kind >= 0)
        hipLaunchKernelGGL(k_output<true>, grid_for(G.nsite, 256), dim3(256), 0, st, G, slicing, ubar, lm, u, m);
    else
        hipLaunchKernelGGL(k_output<false>, grid_for(G.nsite, 256), dim3(256), 0, st, G, slicing, ubar, lm, u, m);
    return hipGetLastError();
}

hipError_t launch_copy_lm(const Geom &G, const double *u0, double *lm, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_lm, grid_for(G.nsite, 256), dim3(256), 0, st, G, u0, lm);
    return hipGetLastError();
}

hipError_t launch_init(const Geom &G, int slicing, const double *u0, double *lm, double *fout, const MatterArg &m,
                       hipStream_t st)
{
    hipError_t e = launch_copy_lm(G, u0, lm, st);
    if (e != hipSuccess) return e;
    const dim3 grid = grid_for(G.nsite, 256), blk(256);
    const bool q9 = G.nq == D2Q9::Q, mat = m.kind >= 0;
    if (q9 && mat)
        hipLaunchKernelGGL((k_init<D2Q9, true>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else if (q9)
        hipLaunchKernelGGL((k_init<D2Q9, false>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else if (mat)
        hipLaunchKernelGGL((k_init<D3Q19, true>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else
        hipLaunchKernelGGL((k_init<D3Q19, false>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    return hipGetLastError();
}

hipError_t launch_gather(const double *fin, const Geom &G, double *f, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_gather<D2Q9>, grid_for(G.nsite, 256), dim3(256), 0, st, fin, G, f);
    else
        hipLaunchKernelGGL(k_gather<D3Q19>, grid_for(G.nsite, 256), dim3(256), 0, st, fin, G, f);
    return hipGetLastError();
}

size_t norm_scratch_doubles(const Geom &G)
{
    return (size_t)((G.nsite + kNormThreads - 1) / kNormThreads) * kFields * 3 + kFields * 3;
}

hipError_t launch_norms(const Geom &G, const double *u, const double *ref, double *scratch, hipStream_t st)
{
    const uint32_t nb = (G.nsite + kNormThreads - 1) / kNormThreads;
    hipLaunchKernelGGL(k_norm_partial, dim3(nb), dim3(kNormThreads), 0, st, G, u, ref, scratch);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kFields), 0, st, scratch, nb, G.nsite,
                       scratch + (size_t)nb * kFields * 3);
    return hipGetLastError();
}

} // namespace lbnr
