// lb_device.h -- device-side building blocks of the Bona-Masso lattice
// Boltzmann step for gfx950.
//
// Everything here is FP64 and written against one fixed evaluation order
// (every contraction sums its index in ascending order; products left to
// right as written; no fused multiply-add, the library is built with
// -ffp-contract=off; IEEE division).  The same order is the one the
// arithmetic definition of the step fixes, so results agree bit for bit
// with any other implementation that follows it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_kernels.h"

namespace lbnr {

constexpr int kFields = 16;

// Lattices (section "Lattice Boltzmann Model"): velocities in the paper's
// column order, upper sign first in every pair; c_s^2 = 1/3 on both.
struct D3Q19 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int cx(int q)
    {
        constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return v[q];
    }
    __host__ __device__ static constexpr int cy(int q)
    {
        constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
        return v[q];
    }
    __host__ __device__ static constexpr int cz(int q)
    {
        constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, -1, 1, 1, -1, -1, 1, 1, -1};
        return v[q];
    }
    // 1/3 (rest), 1/18 (axes), 1/36 (face diagonals)
    __host__ __device__ static constexpr double w(int q)
    {
        return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};

// D2Q9 on a lattice one site thick in z (c_z = 0)
struct D2Q9 {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int cx(int q)
    {
        constexpr int v[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
        return v[q];
    }
    __host__ __device__ static constexpr int cy(int q)
    {
        constexpr int v[Q] = {0, 0, 0, 1, -1, -1, 1, 1, -1};
        return v[q];
    }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    // 4/9 (rest), 1/9 (axes), 1/36 (diagonals)
    __host__ __device__ static constexpr double w(int q)
    {
        return q == 0 ? 4.0 / 9.0 : (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};

// The unqualified names are the D3Q19 set (the z-marching and serving kernels
// are D3Q19 only).
constexpr int kQ = D3Q19::Q;
__host__ __device__ constexpr int cx(int q) { return D3Q19::cx(q); }
__host__ __device__ constexpr int cy(int q) { return D3Q19::cy(q); }
__host__ __device__ constexpr int cz(int q) { return D3Q19::cz(q); }
__host__ __device__ constexpr double wq(int q) { return D3Q19::w(q); }

// symmetric 3x3 storage (xx, xy, xz, yy, yz, zz)
__host__ __device__ constexpr int sidx(int i, int j)
{
    return i == j ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : (i + j == 1 ? 1 : (i + j == 2 ? 2 : 4));
}
__host__ __device__ constexpr int pair_i(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__host__ __device__ constexpr int pair_j(int p) { return p < 3 ? p : (p < 5 ? p - 2 : 2); }

// Inverse of a symmetric 3x3 matrix (a b c / b d e / c e f) from its adjugate.
__device__ __forceinline__ void sym_inverse(const double g[6], double gi[6])
{
    const double a = g[0], b = g[1], c = g[2], d = g[3], e = g[4], f = g[5];
    const double m00 = d * f - e * e;
    const double m01 = c * e - b * f;
    const double m02 = b * e - c * d;
    const double m11 = a * f - c * c;
    const double m12 = b * c - a * e;
    const double m22 = a * d - b * b;
    const double det = a * m00 + b * m01 + c * m02;
    gi[0] = m00 / det;
    gi[1] = m01 / det;
    gi[2] = m02 / det;
    gi[3] = m11 / det;
    gi[4] = m12 / det;
    gi[5] = m22 / det;
}

// gamma^{ij} K_ij over all nine (i, j), i outer
__device__ __forceinline__ double trace_up(const double gi[6], const double K[6])
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += gi[sidx(i, j)] * K[sidx(i, j)];
    return s;
}

// Lapse and metric with their half source (zero shift):
//   R_alpha = -alpha^2 Q,  R_gamma = -2 alpha K,
//   alpha_c = abar + R_alpha/2,  gamma_c = gbar + R_gamma/2.
// ub: the 13 raw moments alpha, gamma[6], K[6].  Out: lm[7] corrected,
// R[7] right-hand sides.
__device__ __forceinline__ void lapse_metric(const double ub[13], int slicing, double lm[7], double R[7])
{
    const double ab = ub[0];
    double gi[6];
    sym_inverse(ub + 1, gi);
    double Q = 0.0;
    if (slicing == kSlicingHarmonic)
        Q = trace_up(gi, ub + 7);
    else if (slicing == kSlicingOnePlusLog)
        Q = trace_up(gi, ub + 7) / ab;
    const double Ra = -(ab * ab * Q);
    R[0] = Ra;
    lm[0] = ab + 0.5 * Ra;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const double Rg = -2.0 * ab * ub[7 + p];
        R[1 + p] = Rg;
        lm[1 + p] = ub[1 + p] + 0.5 * Rg;
    }
}

// Sources of K and V (extrinsic-curvature and momentum-variable equations,
// zero shift; the vacuum part, matter_sources adds the energy-momentum terms)
// at (alpha, gamma, K, V, A, D):  S[6] (pairs i <= j) and Omega[3].  D[k*6 + p] = D_k(ij).  Index conventions: first index of D is
// the derivative index, indices raised with the inverse metric.
__device__ __forceinline__ void bm_sources(double alpha, const double g[6], const double gi[6],
                                           const double K[6], const double V[3],
                                           const double A[3], const double D[18],
                                           double S[6], double Om[3])
{
#define G_(i, j) gi[sidx(i, j)]
#define K_(i, j) K[sidx(i, j)]
#define D_(k, i, j) D[(k) * 6 + sidx(i, j)]
    // K_i^j = g^{jl} K_il
    double Km[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) s += G_(j, l) * K_(i, l);
            Km[i][j] = s;
        }
    double trK = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) trK += Km[i][i];
    double trK2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) trK2 += Km[i][j] * Km[j][i];

    // D_ki^j = g^{jl} D_kil
    double Dm[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < 3; ++l) s += G_(j, l) * D_(k, i, l);
                Dm[k][i][j] = s;
            }
    // D^k_ij = g^{kl} D_lij (symmetric in i, j)
    double Du[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) s += G_(k, l) * D[l * 6 + p];
            Du[k][p] = s;
        }
    // D_k^{ij} = g^{il} D_kl^j
    double Dkk[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < 3; ++l) s += G_(i, l) * Dm[k][l][j];
                Dkk[k][i][j] = s;
            }
    double d1[3], d2[3], d3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) s += Dm[k][i][i];
        d1[k] = s; // D_kr^r
        s = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) s += Du[j][sidx(j, k)];
        d2[k] = s; // D^j_jk
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += Dkk[k][k][r];
        d3[r] = s; // D_k^{kr}
    }
    // Gamma^k_ij = g^{kl} (D_ijl + D_jil - D_lij), symmetric in i, j
    double Ga[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = pair_i(p), j = pair_j(p);
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) s += G_(k, l) * (D_(i, j, l) + D_(j, i, l) - D_(l, i, j));
            Ga[k][p] = s;
        }
#define GA_(k, i, j) Ga[k][sidx(i, j)]
    double gc[3], Au[3], Vu[3], d1u[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += GA_(k, k, r);
        gc[r] = s; // Gamma^k_kr
        s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += G_(r, l) * A[l];
        Au[r] = s;
        s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += G_(r, l) * V[l];
        Vu[r] = s;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += G_(k, l) * d1[l];
        d1u[k] = s; // D^{ks}_s
    }

    // scalar bracket multiplying gamma_ij / 4
    double b1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) b1 += Dkk[k][r][q] * GA_(k, r, q);
    double b2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) b2 += d1[k] * d1u[k];
    double b3 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) b3 += Vu[k] * A[k];
    const double bracket = -b1 + b2 - 2.0 * b3 + trK2 - trK * trK;

#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = pair_i(p), j = pair_j(p);
        double t1 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) t1 += Km[i][k] * K_(k, j);
        t1 = -2.0 * t1;
        const double t2 = trK * K[p];
        double t3 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r) t3 += Dm[i][k][r] * Dm[r][j][k];
        t3 = 2.0 * t3;
        double t4 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r) t4 += Dm[j][k][r] * Dm[r][i][k];
        t4 = 2.0 * t4;
        double t5 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) t5 += gc[r] * Ga[r][p];
        double t6 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r) t6 += GA_(k, r, i) * GA_(r, k, j);
        t6 = -t6;
        double t7 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) t7 += (2.0 * d3[r] - Au[r]) * (D_(i, j, r) + D_(j, i, r));
        t7 = -t7;
        const double t8 = A[i] * (V[j] - 0.5 * d1[j]);
        const double t9 = A[j] * (V[i] - 0.5 * d1[i]);
        double t10 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) t10 += Vu[k] * D[k * 6 + p];
        t10 = -t10;
        const double t11 = 0.25 * g[p] * bracket;
        S[p] = t1 + t2 + t3 + t4 + t5 + t6 + t7 + t8 + t9 + t10 + t11;
    }

#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double o1 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) o1 += A[r] * (r == k ? Km[k][r] - trK : Km[k][r]);
        double o2 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) o2 += (Dm[k][r][q] - 2.0 * Dm[r][k][q]) * Km[q][r];
        double o3 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) o3 += Km[k][r] * (d1[r] - 2.0 * d2[r]);
        Om[k] = alpha * (o1 + o2 - o3);
    }
#undef GA_
#undef D_
#undef K_
#undef G_
}

// Flux of the extrinsic-curvature equation, F^k_ij = alpha lambda^k_ij with
// lambda^k_ij = D^k_ij + 1/2 delta^k_i (A_j + 2 V_j - D_jr^r)
//             + 1/2 delta^k_j (A_i + 2 V_i - D_ir^r) - 1/2 V^k gamma_ij.
// Out: F[k*6 + p].
__device__ __forceinline__ void bm_flux(double alpha, const double g[6], const double gi[6],
                                        const double V[3], const double A[3],
                                        const double D[18], double F[18])
{
    double P[3], Vu[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) t += gi[sidx(i, l)] * D[k * 6 + sidx(i, l)];
            s += t;
        }
        P[k] = A[k] + 2.0 * V[k] - s;
        double v = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) v += gi[sidx(k, l)] * V[l];
        Vu[k] = v;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = pair_i(p), j = pair_j(p);
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) t += gi[sidx(k, l)] * D[l * 6 + p];
            if (k == i) t += 0.5 * P[j];
            if (k == j) t += 0.5 * P[i];
            t -= 0.5 * Vu[k] * g[p];
            F[k * 6 + p] = alpha * t;
        }
}

// Matter (energy-momentum tensor G, units c = 8 pi G = 1) in the sources of
// the extrinsic-curvature and momentum-variable equations (section
// "Bona-Masso evolution equations"), of one of two kinds:
//   kMatterTensor: M = G^00, G^0_k (x, y, z), G_ij (xx, xy, xz, yy, yz, zz);
//   kMatterFluid:  M = (rho, P) of a perfect fluid at rest in the slicing:
//                  alpha^2 G^00 = rho, G^0_k = 0, G_ij = P gamma_ij.
// With R4_ij = G_ij - gamma_ij/2 (-alpha^2 G^00 + tr G), tr G = gamma^{ij} G_ij,
// S_ij gains gamma_ij/4 (2 alpha^2 G^00) - R4_ij (added to the vacuum value
// as one sum) and Omega_k gains alpha (alpha G^0_k).
__device__ __forceinline__ void matter_sources(double alpha, const double g[6], const double gi[6], int kind,
                                               const double M[10], double S[6], double Om[3])
{
    double Gm[6], a2G;
    if (kind == kMatterFluid) {
#pragma unroll
        for (int p = 0; p < 6; ++p) Gm[p] = M[1] * g[p];
        a2G = M[0];
    } else {
#pragma unroll
        for (int p = 0; p < 6; ++p) Gm[p] = M[4 + p];
        a2G = alpha * alpha * M[0];
    }
    const double trG = trace_up(gi, Gm);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const double R4 = Gm[p] - 0.5 * g[p] * (-a2G + trG);
        S[p] += 0.25 * g[p] * (2.0 * a2G) - R4;
    }
    if (kind == kMatterTensor) {
#pragma unroll
        for (int k = 0; k < 3; ++k) Om[k] += alpha * (alpha * M[1 + k]);
    }
}

// c_q . F for the three flux components of one K pair (only the non-zero
// velocity components enter; each direction has at most two).
template <int q, class L = D3Q19>
__device__ __forceinline__ double cdot(double F0, double F1, double F2)
{
    double s = 0.0;
    bool first = true;
    if (L::cx(q) != 0) { s = L::cx(q) > 0 ? F0 : -F0; first = false; }
    if (L::cy(q) != 0) { s = first ? (L::cy(q) > 0 ? F1 : -F1) : (L::cy(q) > 0 ? s + F1 : s - F1); first = false; }
    if (L::cz(q) != 0) { s = first ? (L::cz(q) > 0 ? F2 : -F2) : (L::cz(q) > 0 ? s + F2 : s - F2); first = false; }
    return s;
}

} // namespace lbnr
