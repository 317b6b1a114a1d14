// lb_site.h -- site indexing and pull addressing shared by the kernels
// (periodic lattice, x fastest, one plane of `ps` elements per (field, q)),
// for a lattice L (D3Q19 or D2Q9).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_device.h"
#include "lb_kernels.h"

namespace lbnr {

template <class L>
struct SiteT {
    int x, y, z;
    uint32_t s;                // site index
    uint32_t src[L::Q];        // index of x - c_q (periodic)
};
using Site = SiteT<D3Q19>;

template <class L>
__device__ __forceinline__ bool site_of(const Geom &G, uint32_t s, SiteT<L> &o)
{
    if (s >= G.nsite) return false;
    o.s = s;
    o.x = (int)(s % (uint32_t)G.nx);
    const uint32_t r = s / (uint32_t)G.nx;
    o.y = (int)(r % (uint32_t)G.ny);
    o.z = (int)(r / (uint32_t)G.ny);
    return true;
}

// index of the site at (x + dx, y + dy, z + dz), periodic, |d| <= 1
__device__ __forceinline__ uint32_t neighbour(const Geom &G, int x, int y, int z, int dx, int dy, int dz)
{
    int xx = x + dx, yy = y + dy, zz = z + dz;
    xx = xx < 0 ? xx + G.nx : (xx >= G.nx ? xx - G.nx : xx);
    yy = yy < 0 ? yy + G.ny : (yy >= G.ny ? yy - G.ny : yy);
    zz = zz < 0 ? zz + G.nz : (zz >= G.nz ? zz - G.nz : zz);
    return ((uint32_t)zz * (uint32_t)G.ny + (uint32_t)yy) * (uint32_t)G.nx + (uint32_t)xx;
}

template <class L>
__device__ __forceinline__ void pull_sources(const Geom &G, SiteT<L> &o)
{
#pragma unroll
    for (int q = 0; q < L::Q; ++q) o.src[q] = neighbour(G, o.x, o.y, o.z, -L::cx(q), -L::cy(q), -L::cz(q));
}

template <class L = D3Q19, typename T>
__device__ __forceinline__ T *plane(T *buf, const Geom &G, int F, int q)
{
    return buf + ((size_t)F * L::Q + (size_t)q) * G.ps;
}

// A_k and D_kij at a site from the corrected lapse/metric of its neighbours
template <class L>
__device__ __forceinline__ void stencil(const Geom &G, const SiteT<L> &o, const double *__restrict__ lm,
                                        double alpha, double A[3], double D[18])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t sp = neighbour(G, o.x, o.y, o.z, k == 0, k == 1, k == 2);
        const uint32_t sm = neighbour(G, o.x, o.y, o.z, -(k == 0), -(k == 1), -(k == 2));
        A[k] = (lm[sp] - lm[sm]) / (2.0 * alpha);
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const double *g = lm + (size_t)(1 + p) * G.ps;
            D[k * 6 + p] = (g[sp] - g[sm]) * 0.25;
        }
    }
}

// Per-site collision parameters: corrected fields u[16], right-hand sides
// R[16] and the K flux F[18], from the raw moments and the lapse/metric field.
struct Params {
    double u[kFields];
    double R[kFields];
    double F[18];
};

// matter values at site s (the kind's components; the rest zero)
__device__ __forceinline__ void matter_load(const MatterArg &m, const Geom &G, uint32_t s, double M[10])
{
    const int nc = m.kind == kMatterFluid ? 2 : 10;
#pragma unroll
    for (int c = 0; c < 10; ++c) M[c] = c < nc ? (m.field ? m.field[(size_t)c * G.ps + s] : m.uni[c]) : 0.0;
}

// Collision parameters from the raw moments ub, the corrected lapse/metric c
// with its right-hand sides Rag (lapse_metric(ub)), and the stencil A, D;
// with HasMatter, the matter M of kind mkind enters the sources.
template <bool HasMatter = false>
__device__ __forceinline__ void params_from(const double ub[kFields], const double c[7], const double Rag[7],
                                            const double A[3], const double D[18], Params &P, int mkind = -1,
                                            const double *M = nullptr)
{
#pragma unroll
    for (int F = 0; F < 7; ++F) {
        P.u[F] = c[F];
        P.R[F] = Rag[F];
    }
    const double alpha = c[0];
    double gi[6], S[6], Om[3], V[3];
    sym_inverse(c + 1, gi);
    bm_sources(alpha, c + 1, gi, ub + 7, ub + 13, A, D, S, Om);
    if constexpr (HasMatter) matter_sources(alpha, c + 1, gi, mkind, M, S, Om);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const double RK = alpha * S[p];
        P.R[7 + p] = RK;
        P.u[7 + p] = ub[7 + p] + 0.5 * RK;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.R[13 + k] = Om[k];
        V[k] = ub[13 + k] + 0.5 * Om[k];
        P.u[13 + k] = V[k];
    }
    bm_flux(alpha, c + 1, gi, V, A, D, P.F);
}

template <bool HasMatter = false, class L>
__device__ __forceinline__ void site_params(const Geom &G, const SiteT<L> &o, int slicing,
                                            const double ub[kFields], const double *__restrict__ lm,
                                            Params &P, const MatterArg &m = MatterArg{})
{
    double c[7], Rag[7], A[3], D[18];
    lapse_metric(ub, slicing, c, Rag);
    stencil(G, o, lm, c[0], A, D);
    if constexpr (HasMatter) {
        double M[10];
        matter_load(m, G, o.s, M);
        params_from<true>(ub, c, Rag, A, D, P, m.kind, M);
    } else {
        params_from(ub, c, Rag, A, D, P);
    }
}

} // namespace lbnr
