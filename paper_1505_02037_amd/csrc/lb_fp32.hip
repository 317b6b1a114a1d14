// lb_fp32.hip -- FP32-deviation form of the Bona-Masso lattice Boltzmann step.
//
// Distributions are stored and streamed in FP32 as deviations from the
// rest-state equilibrium, d_q = f_q - w_q u_rest (u_rest: alpha = 1,
// gamma = delta, K = V = 0), halving the bytes per site.  The moments are
// reconstructed in FP64 (u_rest + sum_q d_q), the lapse/metric correction, the
// derivative stencil, the geometry, the sources and the flux stay FP64, and the
// per-direction relaxation runs in FP32 on the deviations:
//   d*_q = d_q - omega (d_q - d^eq_q) + w_q (1 - omega/2) R,
//   d^eq_q = w_q (u - u_rest)                  (alpha, gamma, V)
//          = w_q ((K - 0) + c_q . F / c_s^2)    (K).
// Storage layout, lattices and the two-launch step are those of the FP64 form.
#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"
#include "lb_step.h"

namespace lbnr {

template <class L>
__global__ void __launch_bounds__(256) k_moments32(const float *__restrict__ fin, Geom G, int slicing,
                                                   double *__restrict__ ubar, double *__restrict__ lm)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < G.nsite) moments_site32<L>(fin, G, s, slicing, ubar, lm);
}

template <class L, bool HasMatter, int Coll>
__global__ void __launch_bounds__(256) k_collide32(const float *__restrict__ fin, float *__restrict__ fout, Geom G,
                                                   int slicing, double omega, double srcfac,
                                                   const double *__restrict__ ubar, const double *__restrict__ lm,
                                                   MatterArg m)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < G.nsite) collide_site32<L, HasMatter, Coll>(fin, fout, G, s, slicing, omega, srcfac, ubar, lm, m);
}

// initial deviations: d_q = f^eq_q(u0) - w_q R(u0)/2 - w_q u_rest (FP64, then rounded)
template <int Fld, class L>
__device__ __forceinline__ void init32_field(float *__restrict__ fout, const Geom &G, const SiteT<L> &o,
                                             const Params &P)
{
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
    const double du = P.u[Fld] - urest(Fld);
    const double hR = 0.5 * P.R[Fld];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        double deq;
        if constexpr (isK) {
            const double cF = (double)L::cx(q) * P.F[pk] + (double)L::cy(q) * P.F[6 + pk] +
                              (double)L::cz(q) * P.F[12 + pk];
            deq = L::w(q) * (du + 3.0 * cF);
        } else {
            deq = L::w(q) * du;
        }
        plane<L>(fout, G, Fld, q)[o.src[q]] = (float)(deq - L::w(q) * hR);
    }
    if constexpr (Fld + 1 < kFields) init32_field<Fld + 1>(fout, G, o, P);
}

template <class L, bool HasMatter>
__global__ void __launch_bounds__(256) k_init32(Geom G, int slicing, const double *__restrict__ u0,
                                                const double *__restrict__ lm, float *__restrict__ fout, MatterArg m)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    double u[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) u[F] = u0[(size_t)F * G.nsite + o.s];
    Params P;
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
    pull_sources(G, o);
    init32_field<0>(fout, G, o, P);
}

// distributions of one field at the current time, f = w u_rest + d, FP64
template <class L>
__global__ void __launch_bounds__(256) k_gather32(const float *__restrict__ fin, Geom G, int F, double *__restrict__ f)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    pull_sources(G, o);
    const double ur = urest(F);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        f[(size_t)q * G.nsite + o.s] = L::w(q) * ur + (double)plane<L>(fin, G, F, q)[o.src[q]];
}

static inline dim3 grid32(uint32_t n) { return dim3((n + 255) / 256); }

hipError_t launch_moments32(const float *fin, const Geom &G, int slicing, double *ubar, double *lm, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_moments32<D2Q9>, grid32(G.nsite), dim3(256), 0, st, fin, G, slicing, ubar, lm);
    else
        hipLaunchKernelGGL(k_moments32<D3Q19>, grid32(G.nsite), dim3(256), 0, st, fin, G, slicing, ubar, lm);
    return hipGetLastError();
}

template <class L, bool HasMatter>
static void collide32_instance(int collision, dim3 grid, hipStream_t st, const float *fin, float *fout,
                               const Geom &G, int slicing, double omega, double srcfac, const double *ubar,
                               const double *lm, const MatterArg &m)
{
    if (collision == kCollisionRegularized)
        hipLaunchKernelGGL((k_collide32<L, HasMatter, kCollisionRegularized>), grid, dim3(256), 0, st, fin, fout, G,
                           slicing, omega, srcfac, ubar, lm, m);
    else
        hipLaunchKernelGGL((k_collide32<L, HasMatter, kCollisionBgk>), grid, dim3(256), 0, st, fin, fout, G,
                           slicing, omega, srcfac, ubar, lm, m);
}

hipError_t launch_collide32(const float *fin, float *fout, const Geom &G, int slicing, double omega, double srcfac,
                            const double *ubar, const double *lm, const MatterArg &m, int collision,
                            hipStream_t st)
{
    const dim3 grid = grid32(G.nsite);
    const bool q9 = G.nq == D2Q9::Q, mat = m.kind >= 0;
    if (q9 && mat)
        collide32_instance<D2Q9, true>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else if (q9)
        collide32_instance<D2Q9, false>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else if (mat)
        collide32_instance<D3Q19, true>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    else
        collide32_instance<D3Q19, false>(collision, grid, st, fin, fout, G, slicing, omega, srcfac, ubar, lm, m);
    return hipGetLastError();
}

hipError_t launch_init32(const Geom &G, int slicing, const double *u0, double *lm, float *fout, const MatterArg &m,
                         hipStream_t st)
{
    hipError_t e = launch_copy_lm(G, u0, lm, st);
    if (e != hipSuccess) return e;
    const dim3 grid = grid32(G.nsite), blk(256);
    const bool q9 = G.nq == D2Q9::Q, mat = m.kind >= 0;
    if (q9 && mat)
        hipLaunchKernelGGL((k_init32<D2Q9, true>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else if (q9)
        hipLaunchKernelGGL((k_init32<D2Q9, false>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else if (mat)
        hipLaunchKernelGGL((k_init32<D3Q19, true>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    else
        hipLaunchKernelGGL((k_init32<D3Q19, false>), grid, blk, 0, st, G, slicing, u0, lm, fout, m);
    return hipGetLastError();
}

hipError_t launch_gather32(const float *fin, const Geom &G, int field, double *f, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_gather32<D2Q9>, grid32(G.nsite), dim3(256), 0, st, fin, G, field, f);
    else
        hipLaunchKernelGGL(k_gather32<D3Q19>, grid32(G.nsite), dim3(256), 0, st, fin, G, field, f);
    return hipGetLastError();
}

} // namespace lbnr
