// lb_step.h -- one lattice Boltzmann step at one site, FP64 and FP32-deviation
// forms.  Shared by the single-lattice kernels and the batched serving
// kernels, so both run the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"

namespace lbnr {

// Zeroth moment of field F at a site from its 19 pulled distributions, summed
// plane by plane: the in-plane directions (c_z = 0), those arriving from the
// plane below (c_z = +1), those from the plane above (c_z = -1), each in
// direction order, then (in-plane + below) + above.  The z-marching kernel
// forms the three partial sums in different iterations; every other kernel
// uses the same grouping so that all paths agree bit for bit.
template <typename T>
__device__ __forceinline__ double plane_sum(const T *__restrict__ fin, const Geom &G, int F, const Site &o)
{
    double in_plane = 0.0, below = 0.0, above = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const double f = (double)plane(fin, G, F, q)[o.src[q]];
        if (cz(q) == 0)
            in_plane += f;
        else if (cz(q) > 0)
            below += f;
        else
            above += f;
    }
    return in_plane + below + above;
}

// ---------------------------------------------------------------------------
// FP64 form
// ---------------------------------------------------------------------------

// zeroth moments of all fields at site s and its corrected lapse/metric
__device__ __forceinline__ void moments_site64(const double *__restrict__ fin, const Geom &G, uint32_t s,
                                               int harmonic, double *__restrict__ ubar, double *__restrict__ lm)
{
    Site o;
    site_of(G, s, o);
    pull_sources(G, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) {
        ub[F] = plane_sum<double>(fin, G, F, o);
    }
    double c[7], R[7];
    lapse_metric(ub, harmonic != 0, c, R);
#pragma unroll
    for (int F = 0; F < kFields; ++F) ubar[(size_t)F * G.ps + o.s] = ub[F];
#pragma unroll
    for (int F = 0; F < 7; ++F) lm[(size_t)F * G.ps + o.s] = c[F];
}

// post-collision values of one field's 19 distributions (Eq. numlb with the
// equilibria and sources of the field): out_q = f_q - omega (f_q - feq_q) + S_q
template <int Fld>
__device__ __forceinline__ void relax64(const double fl[kQ], const Params &P, double omega, double srcfac,
                                        double out[kQ])
{
    const double u = P.u[Fld];
    const double hR = srcfac * P.R[Fld];
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        double feq;
        if constexpr (isK) {
            double cF;
            switch (q) {
#define LBNR_CASE(Q_) case Q_: cF = cdot<Q_>(P.F[pk], P.F[6 + pk], P.F[12 + pk]); break;
                LBNR_CASE(0) LBNR_CASE(1) LBNR_CASE(2) LBNR_CASE(3) LBNR_CASE(4) LBNR_CASE(5)
                LBNR_CASE(6) LBNR_CASE(7) LBNR_CASE(8) LBNR_CASE(9) LBNR_CASE(10) LBNR_CASE(11)
                LBNR_CASE(12) LBNR_CASE(13) LBNR_CASE(14) LBNR_CASE(15) LBNR_CASE(16) LBNR_CASE(17)
                LBNR_CASE(18)
#undef LBNR_CASE
            default: cF = 0.0;
            }
            feq = wq(q) * (u + 3.0 * cF);
        } else {
            feq = wq(q) * u;
        }
        const double f = fl[q];
        out[q] = f - omega * (f - feq) + wq(q) * hR;
    }
}

// relax one field's 19 distributions and store them at x
template <int Fld>
__device__ __forceinline__ void collide_field(const double *__restrict__ fin, double *__restrict__ fout,
                                              const Geom &G, const Site &o, const Params &P,
                                              double omega, double srcfac)
{
    double fl[kQ], out[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) fl[q] = plane(fin, G, Fld, q)[o.src[q]];
    relax64<Fld>(fl, P, omega, srcfac, out);
    // streamed: read again only by the next step's pulls
#pragma unroll
    for (int q = 0; q < kQ; ++q) __builtin_nontemporal_store(out[q], &plane(fout, G, Fld, q)[o.s]);
}

template <int Fld>
__device__ __forceinline__ void collide_all(const double *__restrict__ fin, double *__restrict__ fout,
                                            const Geom &G, const Site &o, const Params &P,
                                            double omega, double srcfac)
{
    collide_field<Fld>(fin, fout, G, o, P, omega, srcfac);
    if constexpr (Fld + 1 < kFields) collide_all<Fld + 1>(fin, fout, G, o, P, omega, srcfac);
}

// sources, flux, BGK relaxation with source and pull streaming at site s
__device__ __forceinline__ void collide_site64(const double *__restrict__ fin, double *__restrict__ fout,
                                               const Geom &G, uint32_t s, int harmonic, double omega,
                                               double srcfac, const double *__restrict__ ubar,
                                               const double *__restrict__ lm)
{
    Site o;
    site_of(G, s, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) ub[F] = ubar[(size_t)F * G.ps + o.s];
    Params P;
    site_params(G, o, harmonic, ub, lm, P);
    pull_sources(G, o);
    collide_all<0>(fin, fout, G, o, P, omega, srcfac);
}

// ---------------------------------------------------------------------------
// FP32-deviation form
// ---------------------------------------------------------------------------

__host__ __device__ constexpr double urest(int F) { return (F == 0 || F == 1 || F == 4 || F == 6) ? 1.0 : 0.0; }
__host__ __device__ constexpr float wqf(int q) { return (float)wq(q); }

__device__ __forceinline__ void moments_site32(const float *__restrict__ fin, const Geom &G, uint32_t s,
                                               int harmonic, double *__restrict__ ubar, double *__restrict__ lm)
{
    Site o;
    site_of(G, s, o);
    pull_sources(G, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) {
        ub[F] = urest(F) + plane_sum<float>(fin, G, F, o);
    }
    double c[7], R[7];
    lapse_metric(ub, harmonic != 0, c, R);
#pragma unroll
    for (int F = 0; F < kFields; ++F) ubar[(size_t)F * G.ps + o.s] = ub[F];
#pragma unroll
    for (int F = 0; F < 7; ++F) lm[(size_t)F * G.ps + o.s] = c[F];
}

template <int q>
__device__ __forceinline__ float cdotf(float F0, float F1, float F2)
{
    float s = 0.0f;
    if (cx(q) != 0) s += cx(q) > 0 ? F0 : -F0;
    if (cy(q) != 0) s += cy(q) > 0 ? F1 : -F1;
    if (cz(q) != 0) s += cz(q) > 0 ? F2 : -F2;
    return s;
}

// post-collision deviations of one field's 19 distributions, in FP32:
// out_q = d_q - omega (d_q - d^eq_q) + w_q (1 - omega/2) R
template <int Fld>
__device__ __forceinline__ void relax32(const float fl[kQ], const Params &P, float om, double srcfac, float out[kQ])
{
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
    const float du = (float)(P.u[Fld] - urest(Fld));
    const float hR = (float)(srcfac * P.R[Fld]);
    const float F0 = isK ? (float)P.F[pk] : 0.0f;
    const float F1 = isK ? (float)P.F[6 + pk] : 0.0f;
    const float F2 = isK ? (float)P.F[12 + pk] : 0.0f;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        float deq;
        if constexpr (isK) {
            float cF;
            switch (q) {
#define LBNR_CASE(Q_) case Q_: cF = cdotf<Q_>(F0, F1, F2); break;
                LBNR_CASE(0) LBNR_CASE(1) LBNR_CASE(2) LBNR_CASE(3) LBNR_CASE(4) LBNR_CASE(5)
                LBNR_CASE(6) LBNR_CASE(7) LBNR_CASE(8) LBNR_CASE(9) LBNR_CASE(10) LBNR_CASE(11)
                LBNR_CASE(12) LBNR_CASE(13) LBNR_CASE(14) LBNR_CASE(15) LBNR_CASE(16) LBNR_CASE(17)
                LBNR_CASE(18)
#undef LBNR_CASE
            default: cF = 0.0f;
            }
            deq = wqf(q) * (du + 3.0f * cF);
        } else {
            deq = wqf(q) * du;
        }
        const float d = fl[q];
        out[q] = d - om * (d - deq) + wqf(q) * hR;
    }
}

template <int Fld>
__device__ __forceinline__ void collide32_all(const float *__restrict__ fin, float *__restrict__ fout, const Geom &G,
                                              const Site &o, const Params &P, float om, double srcfac)
{
    float fl[kQ], out[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) fl[q] = plane(fin, G, Fld, q)[o.src[q]];
    relax32<Fld>(fl, P, om, srcfac, out);
#pragma unroll
    for (int q = 0; q < kQ; ++q) __builtin_nontemporal_store(out[q], &plane(fout, G, Fld, q)[o.s]);
    if constexpr (Fld + 1 < kFields) collide32_all<Fld + 1>(fin, fout, G, o, P, om, srcfac);
}

__device__ __forceinline__ void collide_site32(const float *__restrict__ fin, float *__restrict__ fout,
                                               const Geom &G, uint32_t s, int harmonic, double omega,
                                               double srcfac, const double *__restrict__ ubar,
                                               const double *__restrict__ lm)
{
    Site o;
    site_of(G, s, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) ub[F] = ubar[(size_t)F * G.ps + o.s];
    Params P;
    site_params(G, o, harmonic, ub, lm, P);
    pull_sources(G, o);
    collide32_all<0>(fin, fout, G, o, P, (float)omega, srcfac);
}

} // namespace lbnr
