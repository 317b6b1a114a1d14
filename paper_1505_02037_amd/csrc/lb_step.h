// lb_step.h -- one lattice Boltzmann step at one site, FP64 and FP32-deviation
// forms.  Shared by the single-lattice kernels and the batched serving
// kernels, so both run the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"

namespace lbnr {

// One pulled distribution; each is read exactly once per kernel.  FP64 pulls
// are non-temporal loads: in interleaved runs at 256^3 the FP64 step averaged
// ~2 % faster and varied less than with plain loads (the traffic counters read
// ~2 % more fetched bytes); FP32 pulls stay plain loads, which were ~4 %
// faster there.
template <typename T>
__device__ __forceinline__ T pull(const T *p)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Zeroth moment of field F at a site from its pulled distributions, summed
// plane by plane: the in-plane directions (c_z = 0), those arriving from the
// plane below (c_z = +1), those from the plane above (c_z = -1), each in
// direction order, then (in-plane + below) + above.  The z-marching kernel
// forms the three partial sums in different iterations; every other kernel
// uses the same grouping so that all paths agree bit for bit.  (On D2Q9 both
// out-of-plane sums are empty.)
template <typename T, class L>
__device__ __forceinline__ double plane_sum(const T *__restrict__ fin, const Geom &G, int F, const SiteT<L> &o)
{
    double in_plane = 0.0, below = 0.0, above = 0.0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const double f = (double)pull(&plane<L>(fin, G, F, q)[o.src[q]]);
        if (L::cz(q) == 0)
            in_plane += f;
        else if (L::cz(q) > 0)
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
template <class L = D3Q19>
__device__ __forceinline__ void moments_site64(const double *__restrict__ fin, const Geom &G, uint32_t s,
                                               int slicing, double *__restrict__ ubar, double *__restrict__ lm)
{
    SiteT<L> o;
    site_of(G, s, o);
    pull_sources(G, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) {
        ub[F] = plane_sum<double>(fin, G, F, o);
    }
    double c[7], R[7];
    lapse_metric(ub, slicing, c, R);
#pragma unroll
    for (int F = 0; F < kFields; ++F) ubar[(size_t)F * G.ps + o.s] = ub[F];
#pragma unroll
    for (int F = 0; F < 7; ++F) lm[(size_t)F * G.ps + o.s] = c[F];
}

// equilibrium of field Fld in direction q (Eqs. alfa..ekst, zero shift):
// w_q u for the lapse, metric and V; w_q (u + c_q.F / c_s^2) for K
template <class L, int Fld, int q>
__device__ __forceinline__ double feq64(const Params &P)
{
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
    const double u = P.u[Fld];
    if constexpr (isK)
        return L::w(q) * (u + 3.0 * cdot<q, L>(P.F[pk], P.F[6 + pk], P.F[12 + pk]));
    else
        return L::w(q) * u;
}

// post-collision values of one field's distributions (Eq. numlb with the
// equilibria and sources of the field): out_q = f_q - omega (f_q - feq_q) + S_q,
// direction q fixed at compile time
template <class L, int Fld, int q = 0>
__device__ __forceinline__ void relax64_q(const double *fl, const Params &P, double omega, double hR, double *out)
{
    const double feq = feq64<L, Fld, q>(P);
    const double f = fl[q];
    out[q] = f - omega * (f - feq) + L::w(q) * hR;
    if constexpr (q + 1 < L::Q) relax64_q<L, Fld, q + 1>(fl, P, omega, hR, out);
}

template <int Fld, class L = D3Q19>
__device__ __forceinline__ void relax64(const double fl[L::Q], const Params &P, double omega, double srcfac,
                                        double out[L::Q])
{
    relax64_q<L, Fld>(fl, P, omega, srcfac * P.R[Fld], out);
}

// Regularized variant: of the non-equilibrium part f - feq only its zeroth
// and first moments are kept and relaxed as BGK relaxes them,
//   out_q = feq_q + (1 - omega) w_q (m0 + c_q.J / c_s^2) + w_q (1 - omega/2) R,
//   m0 = sum_q (f_q - feq_q),  J = sum_q c_q (f_q - feq_q)   (ascending q).
template <class L, int Fld, int q = 0>
__device__ __forceinline__ void feq64_all(const Params &P, double *feq)
{
    feq[q] = feq64<L, Fld, q>(P);
    if constexpr (q + 1 < L::Q) feq64_all<L, Fld, q + 1>(P, feq);
}

template <class L, int q = 0>
__device__ __forceinline__ void reg_out64(const double *feq, double a, double m0, double J0, double J1, double J2,
                                          double hR, double *out)
{
    out[q] = feq[q] + a * L::w(q) * (m0 + 3.0 * cdot<q, L>(J0, J1, J2)) + L::w(q) * hR;
    if constexpr (q + 1 < L::Q) reg_out64<L, q + 1>(feq, a, m0, J0, J1, J2, hR, out);
}

template <int Fld, class L = D3Q19>
__device__ __forceinline__ void relax64_reg(const double fl[L::Q], const Params &P, double omega, double srcfac,
                                            double out[L::Q])
{
    const double hR = srcfac * P.R[Fld];
    double feq[L::Q];
    feq64_all<L, Fld>(P, feq);
    double m0 = 0.0, J0 = 0.0, J1 = 0.0, J2 = 0.0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const double ne = fl[q] - feq[q];
        m0 += ne;
        if (L::cx(q) != 0) J0 = L::cx(q) > 0 ? J0 + ne : J0 - ne;
        if (L::cy(q) != 0) J1 = L::cy(q) > 0 ? J1 + ne : J1 - ne;
        if (L::cz(q) != 0) J2 = L::cz(q) > 0 ? J2 + ne : J2 - ne;
    }
    reg_out64<L>(feq, 1.0 - omega, m0, J0, J1, J2, hR, out);
}

// relax one field's distributions and store them at x
template <int Fld, class L, int Coll>
__device__ __forceinline__ void collide_field(const double *__restrict__ fin, double *__restrict__ fout,
                                              const Geom &G, const SiteT<L> &o, const Params &P,
                                              double omega, double srcfac)
{
    double fl[L::Q], out[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) fl[q] = pull(&plane<L>(fin, G, Fld, q)[o.src[q]]);
    if constexpr (Coll == kCollisionRegularized)
        relax64_reg<Fld, L>(fl, P, omega, srcfac, out);
    else
        relax64<Fld, L>(fl, P, omega, srcfac, out);
    // streamed: read again only by the next step's pulls
#pragma unroll
    for (int q = 0; q < L::Q; ++q) __builtin_nontemporal_store(out[q], &plane<L>(fout, G, Fld, q)[o.s]);
}

template <int Fld, class L, int Coll>
__device__ __forceinline__ void collide_all(const double *__restrict__ fin, double *__restrict__ fout,
                                            const Geom &G, const SiteT<L> &o, const Params &P,
                                            double omega, double srcfac)
{
    collide_field<Fld, L, Coll>(fin, fout, G, o, P, omega, srcfac);
    if constexpr (Fld + 1 < kFields) collide_all<Fld + 1, L, Coll>(fin, fout, G, o, P, omega, srcfac);
}

// sources, flux, BGK relaxation with source and pull streaming at site s
template <class L = D3Q19, bool HasMatter = false, int Coll = kCollisionBgk>
__device__ __forceinline__ void collide_site64(const double *__restrict__ fin, double *__restrict__ fout,
                                               const Geom &G, uint32_t s, int slicing, double omega,
                                               double srcfac, const double *__restrict__ ubar,
                                               const double *__restrict__ lm, const MatterArg &m = MatterArg{})
{
    SiteT<L> o;
    site_of(G, s, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) ub[F] = ubar[(size_t)F * G.ps + o.s];
    Params P;
    site_params<HasMatter>(G, o, slicing, ub, lm, P, m);
    pull_sources(G, o);
    collide_all<0, L, Coll>(fin, fout, G, o, P, omega, srcfac);
}

// ---------------------------------------------------------------------------
// FP32-deviation form
// ---------------------------------------------------------------------------

__host__ __device__ constexpr double urest(int F) { return (F == 0 || F == 1 || F == 4 || F == 6) ? 1.0 : 0.0; }
template <class L = D3Q19>
__host__ __device__ constexpr float wqf(int q) { return (float)L::w(q); }

template <class L = D3Q19>
__device__ __forceinline__ void moments_site32(const float *__restrict__ fin, const Geom &G, uint32_t s,
                                               int slicing, double *__restrict__ ubar, double *__restrict__ lm)
{
    SiteT<L> o;
    site_of(G, s, o);
    pull_sources(G, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) {
        ub[F] = urest(F) + plane_sum<float>(fin, G, F, o);
    }
    double c[7], R[7];
    lapse_metric(ub, slicing, c, R);
#pragma unroll
    for (int F = 0; F < kFields; ++F) ubar[(size_t)F * G.ps + o.s] = ub[F];
#pragma unroll
    for (int F = 0; F < 7; ++F) lm[(size_t)F * G.ps + o.s] = c[F];
}

template <int q, class L>
__device__ __forceinline__ float cdotf(float F0, float F1, float F2)
{
    float s = 0.0f;
    if (L::cx(q) != 0) s += L::cx(q) > 0 ? F0 : -F0;
    if (L::cy(q) != 0) s += L::cy(q) > 0 ? F1 : -F1;
    if (L::cz(q) != 0) s += L::cz(q) > 0 ? F2 : -F2;
    return s;
}

// post-collision deviations of one field's distributions, in FP32:
// out_q = d_q - omega (d_q - d^eq_q) + w_q (1 - omega/2) R, q fixed at compile time
template <class L, bool isK, int q = 0>
__device__ __forceinline__ void relax32_q(const float *fl, float du, float hR, float F0, float F1, float F2, float om,
                                          float *out)
{
    float deq;
    if constexpr (isK)
        deq = wqf<L>(q) * (du + 3.0f * cdotf<q, L>(F0, F1, F2));
    else
        deq = wqf<L>(q) * du;
    const float d = fl[q];
    out[q] = d - om * (d - deq) + wqf<L>(q) * hR;
    if constexpr (q + 1 < L::Q) relax32_q<L, isK, q + 1>(fl, du, hR, F0, F1, F2, om, out);
}

template <int Fld, class L = D3Q19>
__device__ __forceinline__ void relax32(const float fl[L::Q], const Params &P, float om, double srcfac,
                                        float out[L::Q])
{
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
    const float du = (float)(P.u[Fld] - urest(Fld));
    const float hR = (float)(srcfac * P.R[Fld]);
    const float F0 = isK ? (float)P.F[pk] : 0.0f;
    const float F1 = isK ? (float)P.F[6 + pk] : 0.0f;
    const float F2 = isK ? (float)P.F[12 + pk] : 0.0f;
    relax32_q<L, isK>(fl, du, hR, F0, F1, F2, om, out);
}

// regularized variant in FP32 on the deviations (see relax64_reg)
template <class L, bool isK, int q = 0>
__device__ __forceinline__ void deq32_all(float du, float F0, float F1, float F2, float *deq)
{
    if constexpr (isK)
        deq[q] = wqf<L>(q) * (du + 3.0f * cdotf<q, L>(F0, F1, F2));
    else
        deq[q] = wqf<L>(q) * du;
    if constexpr (q + 1 < L::Q) deq32_all<L, isK, q + 1>(du, F0, F1, F2, deq);
}

template <class L, int q = 0>
__device__ __forceinline__ void reg_out32(const float *deq, float a, float m0, float J0, float J1, float J2, float hR,
                                          float *out)
{
    out[q] = deq[q] + a * wqf<L>(q) * (m0 + 3.0f * cdotf<q, L>(J0, J1, J2)) + wqf<L>(q) * hR;
    if constexpr (q + 1 < L::Q) reg_out32<L, q + 1>(deq, a, m0, J0, J1, J2, hR, out);
}

template <int Fld, class L = D3Q19>
__device__ __forceinline__ void relax32_reg(const float fl[L::Q], const Params &P, float om, double srcfac,
                                            float out[L::Q])
{
    constexpr bool isK = (Fld >= 7 && Fld <= 12);
    constexpr int pk = isK ? Fld - 7 : 0;
    const float du = (float)(P.u[Fld] - urest(Fld));
    const float hR = (float)(srcfac * P.R[Fld]);
    const float F0 = isK ? (float)P.F[pk] : 0.0f;
    const float F1 = isK ? (float)P.F[6 + pk] : 0.0f;
    const float F2 = isK ? (float)P.F[12 + pk] : 0.0f;
    float deq[L::Q];
    deq32_all<L, isK>(du, F0, F1, F2, deq);
    float m0 = 0.0f, J0 = 0.0f, J1 = 0.0f, J2 = 0.0f;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const float ne = fl[q] - deq[q];
        m0 += ne;
        if (L::cx(q) != 0) J0 = L::cx(q) > 0 ? J0 + ne : J0 - ne;
        if (L::cy(q) != 0) J1 = L::cy(q) > 0 ? J1 + ne : J1 - ne;
        if (L::cz(q) != 0) J2 = L::cz(q) > 0 ? J2 + ne : J2 - ne;
    }
    reg_out32<L>(deq, 1.0f - om, m0, J0, J1, J2, hR, out);
}

template <int Fld, class L, int Coll>
__device__ __forceinline__ void collide32_all(const float *__restrict__ fin, float *__restrict__ fout, const Geom &G,
                                              const SiteT<L> &o, const Params &P, float om, double srcfac)
{
    float fl[L::Q], out[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) fl[q] = pull(&plane<L>(fin, G, Fld, q)[o.src[q]]);
    if constexpr (Coll == kCollisionRegularized)
        relax32_reg<Fld, L>(fl, P, om, srcfac, out);
    else
        relax32<Fld, L>(fl, P, om, srcfac, out);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) __builtin_nontemporal_store(out[q], &plane<L>(fout, G, Fld, q)[o.s]);
    if constexpr (Fld + 1 < kFields) collide32_all<Fld + 1, L, Coll>(fin, fout, G, o, P, om, srcfac);
}

template <class L = D3Q19, bool HasMatter = false, int Coll = kCollisionBgk>
__device__ __forceinline__ void collide_site32(const float *__restrict__ fin, float *__restrict__ fout,
                                               const Geom &G, uint32_t s, int slicing, double omega,
                                               double srcfac, const double *__restrict__ ubar,
                                               const double *__restrict__ lm, const MatterArg &m = MatterArg{})
{
    SiteT<L> o;
    site_of(G, s, o);
    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) ub[F] = ubar[(size_t)F * G.ps + o.s];
    Params P;
    site_params<HasMatter>(G, o, slicing, ub, lm, P, m);
    pull_sources(G, o);
    collide32_all<0, L, Coll>(fin, fout, G, o, P, (float)omega, srcfac);
}

} // namespace lbnr
