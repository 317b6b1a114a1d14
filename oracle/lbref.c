/*
 * lbref.c -- FP64 CPU oracle of the lattice Boltzmann step for the Bona-Masso
 * Einstein system.  TEST INFRASTRUCTURE ONLY (see lbref.h).
 *
 * Plain scalar loops over whole-lattice arrays, one pass per stage, so that
 * every stage can be read against the paper:
 *
 *   stage 1  moments      ubar_F = sum_q f_{F,q}            (section "Lattice
 *                                                           Boltzmann Model",
 *                                                           macroscopic moments),
 *            summed plane by plane (in-plane, from below, from above)
 *   stage 2  lapse/metric corrected first: R_alpha = -alpha^2 Q (Eq. alfan,
 *            zero shift), R_gamma = -2 alpha K (three-metric equation, zero
 *            shift), alpha = abar + R_alpha/2, gamma = gbar + R_gamma/2
 *            (macroscopic variables with half source)
 *   stage 3  A_k, D_kij as central differences of the corrected alpha, gamma
 *            (the paper evolves the slicing and the metric first and takes
 *            the derivatives of those; first-order derivative definitions),
 *            then S_ij and Omega_k (extrinsic-curvature and momentum-variable
 *            equations, vacuum, zero shift) at (alpha, gamma, Kbar, Vbar);
 *            R_K = alpha S_ij, R_V = Omega_k; K, V corrected with R/2;
 *            flux alpha lambda^k_ij at the corrected state
 *   stage 4  BGK collision with source (Eq. numlb), equilibria Eqs. alfa..ekst
 *            and sources Eqs. alfa..ekstsor, then streaming with periodic wrap.
 *
 * Arithmetic conventions (fixed so that any other implementation of the same
 * reading can reproduce these numbers exactly):
 *   - every contraction sums its index in ascending order, accumulated from 0;
 *   - products are evaluated left to right as written;
 *   - no fused multiply-add (built with -ffp-contract=off), IEEE division.
 */
#include "lbref.h"

#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 16
#define NQMAX 19

/* D3Q19 velocities in the paper's column order, upper sign first
 * (section "Lattice Boltzmann Model", D3Q19 matrix). */
static const int CQ19[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},
    {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},
    {1, -1, 0}, {-1, 1, 0},
    {1, 1, 0},  {-1, -1, 0},
    {1, 0, -1}, {-1, 0, 1},
    {1, 0, 1},  {-1, 0, -1},
    {0, 1, -1}, {0, -1, 1},
    {0, 1, 1},  {0, -1, -1},
};

/* weights 1/3, 1/18 (axes), 1/36 (face diagonals); c_s^2 = 1/3 */
static const double W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
};

/* D2Q9 velocities in the paper's column order (section "Lattice Boltzmann
 * Model", D2Q9 matrix): c0 = 0, c1,2 = (+-1, 0), c3,4 = (0, +-1),
 * c5,6 = +-(1, -1), c7,8 = +-(1, 1); upper sign first.  c_z = 0. */
static const int CQ9[9][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},
    {0, 1, 0},  {0, -1, 0},
    {1, -1, 0}, {-1, 1, 0},
    {1, 1, 0},  {-1, -1, 0},
};

/* weights 4/9, 1/9 (axes), 1/36 (diagonals); c_s^2 = 1/3 */
static const double W9[9] = {
    4.0 / 9.0,
    1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
};

/* symmetric storage: (xx, xy, xz, yy, yz, zz) */
static const int PAIR_I[6] = {0, 0, 0, 1, 1, 2};
static const int PAIR_J[6] = {0, 1, 2, 1, 2, 2};
static int sym(int i, int j)
{
    static const int S[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return S[i][j];
}

struct lbref {
    int nq;                 /* 19 (D3Q19) or 9 (D2Q9) */
    const int (*cq)[3];     /* velocities */
    const double *w;        /* weights */
    int nx, ny, nz;
    size_t nsite;
    double tau, omega, srcfac;
    int slicing;
    int collision; /* LBREF_COLLISION_BGK or LBREF_COLLISION_REGULARIZED */
    long long nstep;
    double *f;     /* [NF][nq][nsite] current distributions */
    double *fpost; /* [NF][nq][nsite] post-collision scratch */
    double *ubar;  /* [NF][nsite] zeroth moments */
    double *ucor;  /* [NF][nsite] moments with half source */
    double *R;     /* [NF][nsite] right-hand sides */
    double *flux;  /* [3][6][nsite] alpha lambda^k_(ij) */
    int matter;      /* 0: vacuum; 1: the same values at every site; 2: values per site */
    int matter_kind; /* LBREF_MATTER_TENSOR (10 values) or LBREF_MATTER_FLUID (rho, P) */
    double matter_uniform[10];
    double *matter_field; /* [ncomp][nsite] when matter == 2 */
};

static int matter_ncomp(int kind) { return kind == LBREF_MATTER_FLUID ? 2 : 10; }

/* the matter values at site c (NULL in vacuum) */
static const double *matter_at(const lbref *h, size_t c, double M[10])
{
    if (h->matter == 0) return NULL;
    if (h->matter == 1) return h->matter_uniform;
    for (int m = 0; m < matter_ncomp(h->matter_kind); ++m) M[m] = h->matter_field[(size_t)m * h->nsite + c];
    return M;
}

static size_t site_index(const lbref *h, int x, int y, int z)
{
    return ((size_t)z * (size_t)h->ny + (size_t)y) * (size_t)h->nx + (size_t)x;
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* ------------------------------------------------------------------------ */
/* 3x3 algebra                                                              */
/* ------------------------------------------------------------------------ */

static void full3(const double s[6], double m[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = s[sym(i, j)];
}

/* inverse of a symmetric 3x3 matrix through its adjugate */
static void inv3(const double g[6], double gi[3][3])
{
    const double a = g[0], b = g[1], c = g[2], d = g[3], e = g[4], f = g[5];
    const double axx = d * f - e * e;
    const double axy = c * e - b * f;
    const double axz = b * e - c * d;
    const double ayy = a * f - c * c;
    const double ayz = b * c - a * e;
    const double azz = a * d - b * b;
    const double det = a * axx + b * axy + c * axz;
    gi[0][0] = axx / det;
    gi[0][1] = axy / det;
    gi[0][2] = axz / det;
    gi[1][1] = ayy / det;
    gi[1][2] = ayz / det;
    gi[2][2] = azz / det;
    gi[1][0] = gi[0][1];
    gi[2][0] = gi[0][2];
    gi[2][1] = gi[1][2];
}

/* tr K = gamma^{ij} K_ij, summed over i then j */
static double trace_up(const double gi[3][3], const double K[3][3])
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += gi[i][j] * K[i][j];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Bona-Masso right-hand sides (vacuum, zero shift)                         */
/* ------------------------------------------------------------------------ */

/*
 * Matter part of the sources (section "Bona-Masso evolution equations", the
 * energy-momentum terms of S_ij and Omega_k; units c = 8 pi G = 1).
 *   kind 0 (tensor): M holds G^00, G^0_k (k = x, y, z), G_ij (xx, xy, xz,
 *          yy, yz, zz);
 *   kind 1 (perfect fluid at rest in the slicing, section "Expansion of flat
 *          universe"): M holds rho and P, and G^00 = rho / alpha^2,
 *          G^0_k = 0, G_ij = P gamma_ij at the site's lapse and metric.
 * With R4_ij = G_ij - gamma_ij/2 (-alpha^2 G^00 + tr G), tr G = gamma^{ij} G_ij,
 * S_ij gains -R4_ij and gamma_ij/4 (2 alpha^2 G^00) from its bracket, and
 * Omega_k gains alpha (alpha G^0_k).  The matter part is added after the
 * vacuum part, as one sum per component:
 *   S_ij += gamma_ij/4 (2 alpha^2 G^00) - R4_ij,  Omega_k += alpha (alpha G^0_k)
 * (for the fluid alpha^2 G^00 is rho itself and Omega_k is unchanged).
 */
static void matter_sources(double alpha, const double gi[3][3], const double g[3][3], int kind,
                           const double *M, double S6[6], double Om[3])
{
    double Gm[3][3];
    double a2G;
    if (kind == 1) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Gm[i][j] = M[1] * g[i][j];
        a2G = M[0];
    } else {
        full3(M + 4, Gm);
        a2G = alpha * alpha * M[0];
    }
    const double trG = trace_up(gi, Gm);
    for (int p = 0; p < 6; ++p) {
        const int i = PAIR_I[p], j = PAIR_J[p];
        const double R4 = Gm[i][j] - 0.5 * g[i][j] * (-a2G + trG);
        S6[p] += 0.25 * g[i][j] * (2.0 * a2G) - R4;
    }
    if (kind == 0)
        for (int k = 0; k < 3; ++k) Om[k] += alpha * (alpha * M[1 + k]);
}

/*
 * S_ij and Omega_k from the extrinsic-curvature and momentum-variable
 * equations with B = 0 (zero shift); the matter part (G) is added by
 * matter_sources when a matter field is set.  Index conventions: the first index of D is
 * the derivative index; indices are raised with the inverse 3-metric.
 *   K_i^j = g^{jl} K_il          D^k_ij = g^{kl} D_lij     D_ki^j = g^{jl} D_kil
 *   D_k^{ij} = g^{il} D_kl^j     D_kr^r, D^j_jk, D_k^{kr} their traces
 *   Gamma^k_ij = g^{kl} (D_ijl + D_jil - D_lij)   (Christoffel symbols with
 *   D = d gamma / 2)
 * S is evaluated for the six pairs i <= j only.
 */
static void bm_sources(double alpha, const double gi[3][3], const double g[3][3],
                       const double K[3][3], const double V[3], const double A[3],
                       const double D[3][3][3], int mkind, const double *M, double S6[6], double Om[3])
{
    double Kmix[3][3], Dup[3][3][3], Dmix[3][3][3], Dkup[3][3][3], Gam[3][3][3];
    double d1[3], d2[3], d3[3], gc[3], Au[3], Vu[3];
    double trK, trK2, s;

    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            s = 0.0;
            for (int l = 0; l < 3; ++l) s += gi[j][l] * K[i][l];
            Kmix[i][j] = s;
        }
    trK = 0.0;
    for (int i = 0; i < 3; ++i) trK += Kmix[i][i];
    trK2 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) trK2 += Kmix[i][j] * Kmix[j][i];

    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                s = 0.0;
                for (int l = 0; l < 3; ++l) s += gi[k][l] * D[l][i][j];
                Dup[k][i][j] = s;
            }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                s = 0.0;
                for (int l = 0; l < 3; ++l) s += gi[j][l] * D[k][i][l];
                Dmix[k][i][j] = s;
            }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                s = 0.0;
                for (int l = 0; l < 3; ++l) s += gi[i][l] * Dmix[k][l][j];
                Dkup[k][i][j] = s;
            }
    for (int k = 0; k < 3; ++k) {
        s = 0.0;
        for (int i = 0; i < 3; ++i) s += Dmix[k][i][i];
        d1[k] = s; /* D_kr^r */
    }
    for (int k = 0; k < 3; ++k) {
        s = 0.0;
        for (int j = 0; j < 3; ++j) s += Dup[j][j][k];
        d2[k] = s; /* D^j_jk */
    }
    for (int r = 0; r < 3; ++r) {
        s = 0.0;
        for (int k = 0; k < 3; ++k) s += Dkup[k][k][r];
        d3[r] = s; /* D_k^{kr} */
    }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                s = 0.0;
                for (int l = 0; l < 3; ++l)
                    s += gi[k][l] * (D[i][j][l] + D[j][i][l] - D[l][i][j]);
                Gam[k][i][j] = s;
            }
    for (int r = 0; r < 3; ++r) {
        s = 0.0;
        for (int k = 0; k < 3; ++k) s += Gam[k][k][r];
        gc[r] = s; /* Gamma^k_kr */
    }
    for (int r = 0; r < 3; ++r) {
        s = 0.0;
        for (int l = 0; l < 3; ++l) s += gi[r][l] * A[l];
        Au[r] = s;
        s = 0.0;
        for (int l = 0; l < 3; ++l) s += gi[r][l] * V[l];
        Vu[r] = s;
    }

    /* scalar bracket multiplying gamma_ij / 4 */
    double b1 = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) b1 += Dkup[k][r][q] * Gam[k][r][q];
    /* D_kr^r D^{ks}_s: the second factor is the metric trace D_sr^r with its
     * free index raised (the printed index placement D_s^{ks} does not make
     * the exact vacuum solutions satisfy the equation; see the reading in the
     * design notes) */
    double d1u[3];
    for (int k = 0; k < 3; ++k) {
        s = 0.0;
        for (int l = 0; l < 3; ++l) s += gi[k][l] * d1[l];
        d1u[k] = s;
    }
    double b2 = 0.0;
    for (int k = 0; k < 3; ++k) b2 += d1[k] * d1u[k];
    double b3 = 0.0;
    for (int k = 0; k < 3; ++k) b3 += Vu[k] * A[k];
    const double bracket = -b1 + b2 - 2.0 * b3 + trK2 - trK * trK;

    for (int p = 0; p < 6; ++p) {
        const int i = PAIR_I[p], j = PAIR_J[p];
        double t1 = 0.0; /* K_i^k K_kj */
        for (int k = 0; k < 3; ++k) t1 += Kmix[i][k] * K[k][j];
        t1 = -2.0 * t1;
        const double t2 = trK * K[i][j];
        double t3 = 0.0; /* D_ik^r D_rj^k */
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) t3 += Dmix[i][k][r] * Dmix[r][j][k];
        t3 = 2.0 * t3;
        double t4 = 0.0; /* D_jk^r D_ri^k */
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) t4 += Dmix[j][k][r] * Dmix[r][i][k];
        t4 = 2.0 * t4;
        double t5 = 0.0; /* Gamma^k_kr Gamma^r_ij */
        for (int r = 0; r < 3; ++r) t5 += gc[r] * Gam[r][i][j];
        double t6 = 0.0; /* Gamma^k_ri Gamma^r_kj */
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) t6 += Gam[k][r][i] * Gam[r][k][j];
        t6 = -t6;
        double t7 = 0.0; /* (2 D_k^{kr} - A^r)(D_ijr + D_jir) */
        for (int r = 0; r < 3; ++r) t7 += (2.0 * d3[r] - Au[r]) * (D[i][j][r] + D[j][i][r]);
        t7 = -t7;
        const double t8 = A[i] * (V[j] - 0.5 * d1[j]);
        const double t9 = A[j] * (V[i] - 0.5 * d1[i]);
        double t10 = 0.0; /* V^k D_kij */
        for (int k = 0; k < 3; ++k) t10 += Vu[k] * D[k][i][j];
        t10 = -t10;
        const double t11 = 0.25 * g[i][j] * bracket;
        S6[p] = t1 + t2 + t3 + t4 + t5 + t6 + t7 + t8 + t9 + t10 + t11;
    }

    for (int k = 0; k < 3; ++k) {
        double o1 = 0.0; /* A_r (K^r_k - tr K delta^r_k) */
        for (int r = 0; r < 3; ++r) o1 += A[r] * (Kmix[k][r] - (r == k ? trK : 0.0));
        double o2 = 0.0; /* (D_kr^s - 2 D_rk^s) K^r_s */
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) o2 += (Dmix[k][r][q] - 2.0 * Dmix[r][k][q]) * Kmix[q][r];
        double o3 = 0.0; /* K^r_k (D_rs^s - 2 D^j_jr) */
        for (int r = 0; r < 3; ++r) o3 += Kmix[k][r] * (d1[r] - 2.0 * d2[r]);
        Om[k] = alpha * (o1 + o2 - o3);
    }
    if (M) matter_sources(alpha, gi, g, mkind, M, S6, Om);
}

/*
 * lambda^k_ij = D^k_ij + 1/2 delta^k_i (A_j + 2 V_j - D_jr^r)
 *             + 1/2 delta^k_j (A_i + 2 V_i - D_ir^r) - 1/2 V^k gamma_ij
 * (flux of the extrinsic-curvature equation); out: lam[k][pair].
 */
static void bm_lambda(const double gi[3][3], const double g[3][3], const double V[3],
                      const double A[3], const double D[3][3][3], double lam[3][6])
{
    double Dup[3][3][3], d1[3], Vu[3], P[3], s;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                s = 0.0;
                for (int l = 0; l < 3; ++l) s += gi[k][l] * D[l][i][j];
                Dup[k][i][j] = s;
            }
    for (int k = 0; k < 3; ++k) {
        s = 0.0;
        for (int i = 0; i < 3; ++i) {
            double t = 0.0; /* D_ki^i = g^{il} D_kil */
            for (int l = 0; l < 3; ++l) t += gi[i][l] * D[k][i][l];
            s += t;
        }
        d1[k] = s;
        s = 0.0;
        for (int l = 0; l < 3; ++l) s += gi[k][l] * V[l];
        Vu[k] = s;
    }
    for (int j = 0; j < 3; ++j) P[j] = A[j] + 2.0 * V[j] - d1[j];
    for (int k = 0; k < 3; ++k)
        for (int p = 0; p < 6; ++p) {
            const int i = PAIR_I[p], j = PAIR_J[p];
            double t = Dup[k][i][j];
            if (k == i) t += 0.5 * P[j];
            if (k == j) t += 0.5 * P[i];
            t -= 0.5 * Vu[k] * g[i][j];
            lam[k][p] = t;
        }
}

/* ------------------------------------------------------------------------ */
/* Lattice stages                                                           */
/* ------------------------------------------------------------------------ */

#define FLD(arr, F, n) ((arr) + (size_t)(F) * (n))
#define DIST(arr, F, q, n) ((arr) + ((size_t)(F) * (size_t)h->nq + (size_t)(q)) * (n))

/* stage 1: ubar_F = sum_q f_{F,q} */
/* The sum over the directions is taken plane by plane: the directions
 * lying in the site's z-plane (c_z = 0), those arriving from the plane below
 * (c_z = +1), those arriving from the plane above (c_z = -1), each in index
 * order, then (in-plane + below) + above. */
static void stage_moments(lbref *h)
{
    const size_t n = h->nsite;
#pragma omp parallel for schedule(static)
    for (long long ss = 0; ss < (long long)n; ++ss) {
        const size_t x = (size_t)ss;
        for (int F = 0; F < NF; ++F) {
            double in_plane = 0.0, below = 0.0, above = 0.0;
            for (int q = 0; q < h->nq; ++q) {
                const double f = DIST(h->f, F, q, n)[x];
                if (h->cq[q][2] == 0)
                    in_plane += f;
                else if (h->cq[q][2] > 0)
                    below += f;
                else
                    above += f;
            }
            FLD(h->ubar, F, n)[x] = in_plane + below + above;
        }
    }
}

/* stage 2: local half-source correction of alpha and gamma */
static void stage_lapse_metric(lbref *h, const double *ubar, double *ucor, double *R)
{
    const size_t n = h->nsite;
#pragma omp parallel for schedule(static)
    for (long long ss = 0; ss < (long long)n; ++ss) {
        const size_t x = (size_t)ss;
        double gb[6], Kb6[6], gi[3][3], Kb[3][3];
        const double ab = FLD(ubar, 0, n)[x];
        for (int p = 0; p < 6; ++p) {
            gb[p] = FLD(ubar, 1 + p, n)[x];
            Kb6[p] = FLD(ubar, 7 + p, n)[x];
        }
        full3(Kb6, Kb);
        inv3(gb, gi);
        double Q = 0.0; /* section "Gauge choices" */
        if (h->slicing == LBREF_SLICING_HARMONIC)
            Q = trace_up(gi, Kb);
        else if (h->slicing == LBREF_SLICING_ONE_PLUS_LOG)
            Q = trace_up(gi, Kb) / ab;
        const double Ra = -(ab * ab * Q);
        FLD(R, 0, n)[x] = Ra;
        FLD(ucor, 0, n)[x] = ab + 0.5 * Ra;
        for (int p = 0; p < 6; ++p) {
            const double Rg = -2.0 * ab * Kb6[p];
            FLD(R, 1 + p, n)[x] = Rg;
            FLD(ucor, 1 + p, n)[x] = gb[p] + 0.5 * Rg;
        }
    }
}

/* A_k and D_kij at site (x,y,z) from the lapse/metric array lm (fields 0..6) */
static void stencil(const lbref *h, const double *lm, int x, int y, int z,
                    double A[3], double D[3][3][3])
{
    const size_t n = h->nsite;
    const size_t c = site_index(h, x, y, z);
    const double a = FLD(lm, 0, n)[c];
    for (int k = 0; k < 3; ++k) {
        const int dx = (k == 0), dy = (k == 1), dz = (k == 2);
        const size_t sp = site_index(h, wrap(x + dx, h->nx), wrap(y + dy, h->ny), wrap(z + dz, h->nz));
        const size_t sm = site_index(h, wrap(x - dx, h->nx), wrap(y - dy, h->ny), wrap(z - dz, h->nz));
        A[k] = (FLD(lm, 0, n)[sp] - FLD(lm, 0, n)[sm]) / (2.0 * a);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const int p = sym(i, j);
                D[k][i][j] = (FLD(lm, 1 + p, n)[sp] - FLD(lm, 1 + p, n)[sm]) * 0.25;
            }
    }
}

/*
 * Per-site part of stage 3.  lm holds the lapse and metric (fields 0..6) the
 * derivatives and geometry are taken from; kv holds K and V (fields 7..15) at
 * which the sources are evaluated.  With halfstep = 1 (time step) K and V are
 * corrected by R/2 and the flux uses the corrected V; with halfstep = 0
 * (initialisation at u0) K and V are used as given.
 */
static void site_curvature(const lbref *h, const double *lm, const double *kv,
                           int x, int y, int z, int halfstep,
                           double RK[6], double Om[3], double Kc[6], double Vc[3],
                           double lam_alpha[3][6])
{
    const size_t n = h->nsite;
    const size_t c = site_index(h, x, y, z);
    double A[3], D[3][3][3], g6[6], g[3][3], gi[3][3], Kb6[6], Kb[3][3];
    double Vb[3], S6[6], lam[3][6];
    stencil(h, lm, x, y, z, A, D);
    const double alpha = FLD(lm, 0, n)[c];
    for (int p = 0; p < 6; ++p) {
        g6[p] = FLD(lm, 1 + p, n)[c];
        Kb6[p] = FLD(kv, 7 + p, n)[c];
    }
    for (int k = 0; k < 3; ++k) Vb[k] = FLD(kv, 13 + k, n)[c];
    full3(g6, g);
    full3(Kb6, Kb);
    inv3(g6, gi);
    double M[10];
    bm_sources(alpha, gi, g, Kb, Vb, A, D, h->matter_kind, matter_at(h, c, M), S6, Om);
    for (int p = 0; p < 6; ++p) {
        RK[p] = alpha * S6[p];
        Kc[p] = halfstep ? Kb6[p] + 0.5 * RK[p] : Kb6[p];
    }
    for (int k = 0; k < 3; ++k) Vc[k] = halfstep ? Vb[k] + 0.5 * Om[k] : Vb[k];
    bm_lambda(gi, g, Vc, A, D, lam);
    for (int k = 0; k < 3; ++k)
        for (int p = 0; p < 6; ++p) lam_alpha[k][p] = alpha * lam[k][p];
}

/*
 * stage 3 over the lattice: derivatives of the corrected lapse/metric,
 * sources of K and V at (alpha, gamma, Kbar, Vbar), half-source correction of
 * K and V, and the flux alpha lambda at the corrected state.
 */
static void stage_curvature(lbref *h)
{
    const size_t n = h->nsite;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < h->nz; ++z)
        for (int y = 0; y < h->ny; ++y)
            for (int x = 0; x < h->nx; ++x) {
                const size_t c = site_index(h, x, y, z);
                double RK[6], Om[3], Kc[6], Vc[3], fl[3][6];
                site_curvature(h, h->ucor, h->ubar, x, y, z, 1, RK, Om, Kc, Vc, fl);
                for (int p = 0; p < 6; ++p) {
                    FLD(h->R, 7 + p, n)[c] = RK[p];
                    FLD(h->ucor, 7 + p, n)[c] = Kc[p];
                }
                for (int k = 0; k < 3; ++k) {
                    FLD(h->R, 13 + k, n)[c] = Om[k];
                    FLD(h->ucor, 13 + k, n)[c] = Vc[k];
                }
                for (int k = 0; k < 3; ++k)
                    for (int p = 0; p < 6; ++p) FLD(h->flux, k * 6 + p, n)[c] = fl[k][p];
            }
}

/* equilibrium of field F in direction q at site c (Eqs. alfa..ekst, zero shift) */
static double feq_at(const lbref *h, int F, int q, size_t c)
{
    const size_t n = h->nsite;
    const double u = FLD(h->ucor, F, n)[c];
    if (F >= 7 && F <= 12) {
        const int p = F - 7;
        double cF = 0.0;
        for (int m = 0; m < 3; ++m) cF += (double)h->cq[q][m] * FLD(h->flux, m * 6 + p, n)[c];
        return h->w[q] * (u + 3.0 * cF); /* 1/c_s^2 = 3 */
    }
    return h->w[q] * u;
}

/* stage 4: BGK collision with source (Eq. numlb), or its regularized
 * variant, then periodic streaming */
static void stage_collide_stream(lbref *h)
{
    const size_t n = h->nsite;
    const double omega = h->omega, srcfac = h->srcfac;
#pragma omp parallel for schedule(static)
    for (long long ss = 0; ss < (long long)n; ++ss) {
        const size_t c = (size_t)ss;
        for (int F = 0; F < NF; ++F) {
            const double hR = srcfac * FLD(h->R, F, n)[c];
            if (h->collision == LBREF_COLLISION_REGULARIZED) {
                /* the non-equilibrium part keeps only its zeroth and first
                 * moments, m0 = sum_q (f - feq) and J = sum_q c_q (f - feq),
                 * and relaxes them as BGK does: f* = feq + (1 - omega) w
                 * (m0 + c.J / c_s^2) + w (1 - omega/2) R */
                double m0 = 0.0, J[3] = {0.0, 0.0, 0.0};
                for (int q = 0; q < h->nq; ++q) {
                    const double ne = DIST(h->f, F, q, n)[c] - feq_at(h, F, q, c);
                    m0 += ne;
                    for (int m = 0; m < 3; ++m) J[m] += (double)h->cq[q][m] * ne;
                }
                for (int q = 0; q < h->nq; ++q) {
                    double cJ = 0.0;
                    for (int m = 0; m < 3; ++m) cJ += (double)h->cq[q][m] * J[m];
                    DIST(h->fpost, F, q, n)[c] =
                        feq_at(h, F, q, c) + (1.0 - omega) * h->w[q] * (m0 + 3.0 * cJ) + h->w[q] * hR;
                }
                continue;
            }
            for (int q = 0; q < h->nq; ++q) {
                const double f = DIST(h->f, F, q, n)[c];
                const double feq = feq_at(h, F, q, c);
                const double src = h->w[q] * hR;
                DIST(h->fpost, F, q, n)[c] = f - omega * (f - feq) + src;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < h->nz; ++z)
        for (int F = 0; F < NF; ++F)
            for (int q = 0; q < h->nq; ++q)
                for (int y = 0; y < h->ny; ++y)
                    for (int x = 0; x < h->nx; ++x) {
                        const size_t src = site_index(h, wrap(x - h->cq[q][0], h->nx),
                                                      wrap(y - h->cq[q][1], h->ny),
                                                      wrap(z - h->cq[q][2], h->nz));
                        DIST(h->f, F, q, n)[site_index(h, x, y, z)] = DIST(h->fpost, F, q, n)[src];
                    }
}

/* ------------------------------------------------------------------------ */
/* API                                                                      */
/* ------------------------------------------------------------------------ */

int lbref_create(int nx, int ny, int nz, double tau, int slicing, lbref **out)
{
    return lbref_create_lattice(LBREF_D3Q19, nx, ny, nz, tau, slicing, out);
}

int lbref_create_lattice(int lattice, int nx, int ny, int nz, double tau, int slicing, lbref **out)
{
    if (!out) return LBREF_EINVAL;
    *out = NULL;
    if (lattice != LBREF_D3Q19 && lattice != LBREF_D2Q9) return LBREF_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return LBREF_EINVAL;
    if (lattice == LBREF_D2Q9 && nz != 1) return LBREF_EINVAL;
    if (!(tau > 0.5)) return LBREF_EINVAL;
    if (slicing != LBREF_SLICING_HARMONIC && slicing != LBREF_SLICING_GEODESIC &&
        slicing != LBREF_SLICING_ONE_PLUS_LOG)
        return LBREF_EINVAL;
    lbref *h = (lbref *)calloc(1, sizeof(lbref));
    if (!h) return LBREF_ENOMEM;
    h->nq = lattice;
    h->cq = lattice == LBREF_D2Q9 ? CQ9 : CQ19;
    h->w = lattice == LBREF_D2Q9 ? W9 : W19;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->nsite = (size_t)nx * (size_t)ny * (size_t)nz;
    h->tau = tau;
    h->omega = 1.0 / tau;
    h->srcfac = 1.0 - 0.5 * h->omega; /* (1 - dt/(2 tau)) */
    h->slicing = slicing;
    const size_t n = h->nsite;
    h->f = (double *)calloc(n * NF * (size_t)h->nq, sizeof(double));
    h->fpost = (double *)calloc(n * NF * (size_t)h->nq, sizeof(double));
    h->ubar = (double *)calloc(n * NF, sizeof(double));
    h->ucor = (double *)calloc(n * NF, sizeof(double));
    h->R = (double *)calloc(n * NF, sizeof(double));
    h->flux = (double *)calloc(n * 18, sizeof(double));
    if (!h->f || !h->fpost || !h->ubar || !h->ucor || !h->R || !h->flux) {
        lbref_destroy(h);
        return LBREF_ENOMEM;
    }
    *out = h;
    return LBREF_OK;
}

void lbref_destroy(lbref *h)
{
    if (!h) return;
    free(h->f);
    free(h->fpost);
    free(h->ubar);
    free(h->ucor);
    free(h->R);
    free(h->flux);
    free(h->matter_field);
    free(h);
}

int lbref_init_fields(lbref *h, const double *u0)
{
    if (!h || !u0) return LBREF_EINVAL;
    const size_t n = h->nsite;
    /* Every quantity is evaluated at u0: the right-hand sides R(u0), the
     * derivatives of the u0 lapse/metric and the flux at u0.  Then
     * f_q = f^eq_q(u0) - w_q R(u0)/2, so that sum_q f + R/2 = u0. */
    memcpy(h->ubar, u0, n * NF * sizeof(double));
    memcpy(h->ucor, u0, n * NF * sizeof(double));
    {
        double *scratch = (double *)malloc(n * NF * sizeof(double));
        if (!scratch) return LBREF_ENOMEM;
        /* R_alpha, R_gamma at u0 (the corrected values it also writes are
         * discarded: ucor keeps u0) */
        stage_lapse_metric(h, h->ubar, scratch, h->R);
        free(scratch);
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < h->nz; ++z)
        for (int y = 0; y < h->ny; ++y)
            for (int x = 0; x < h->nx; ++x) {
                const size_t c = site_index(h, x, y, z);
                double RK[6], Om[3], Kc[6], Vc[3], fl[3][6];
                site_curvature(h, h->ubar, h->ubar, x, y, z, 0, RK, Om, Kc, Vc, fl);
                for (int p = 0; p < 6; ++p) FLD(h->R, 7 + p, n)[c] = RK[p];
                for (int k = 0; k < 3; ++k) FLD(h->R, 13 + k, n)[c] = Om[k];
                for (int k = 0; k < 3; ++k)
                    for (int p = 0; p < 6; ++p) FLD(h->flux, k * 6 + p, n)[c] = fl[k][p];
            }
#pragma omp parallel for schedule(static)
    for (long long ss = 0; ss < (long long)n; ++ss) {
        const size_t c = (size_t)ss;
        for (int F = 0; F < NF; ++F) {
            const double hR = 0.5 * FLD(h->R, F, n)[c];
            for (int q = 0; q < h->nq; ++q)
                DIST(h->f, F, q, n)[c] = feq_at(h, F, q, c) - h->w[q] * hR;
        }
    }
    h->nstep = 0;
    return LBREF_OK;
}

int lbref_step(lbref *h, long long nsteps)
{
    if (!h || nsteps < 0) return LBREF_EINVAL;
    for (long long s = 0; s < nsteps; ++s) {
        stage_moments(h);
        stage_lapse_metric(h, h->ubar, h->ucor, h->R);
        stage_curvature(h);
        stage_collide_stream(h);
        h->nstep++;
    }
    return LBREF_OK;
}

int lbref_moments(lbref *h, double *u_out)
{
    if (!h || !u_out) return LBREF_EINVAL;
    stage_moments(h);
    stage_lapse_metric(h, h->ubar, h->ucor, h->R);
    stage_curvature(h);
    memcpy(u_out, h->ucor, h->nsite * NF * sizeof(double));
    return LBREF_OK;
}

int lbref_get_distributions(const lbref *h, double *f_out)
{
    if (!h || !f_out) return LBREF_EINVAL;
    memcpy(f_out, h->f, h->nsite * NF * (size_t)h->nq * sizeof(double));
    return LBREF_OK;
}

int lbref_set_distributions(lbref *h, const double *f_in)
{
    if (!h || !f_in) return LBREF_EINVAL;
    memcpy(h->f, f_in, h->nsite * NF * (size_t)h->nq * sizeof(double));
    return LBREF_OK;
}

long long lbref_nsteps_done(const lbref *h) { return h ? h->nstep : -1; }

int lbref_set_collision(lbref *h, int kind)
{
    if (!h || (kind != LBREF_COLLISION_BGK && kind != LBREF_COLLISION_REGULARIZED)) return LBREF_EINVAL;
    h->collision = kind;
    return LBREF_OK;
}

int lbref_set_matter(lbref *h, int kind, const double *M, int per_site)
{
    if (!h) return LBREF_EINVAL;
    if (kind != LBREF_MATTER_TENSOR && kind != LBREF_MATTER_FLUID) return LBREF_EINVAL;
    if (!M) {
        h->matter = 0;
        return LBREF_OK;
    }
    const int nc = matter_ncomp(kind);
    if (per_site) {
        if (!h->matter_field) {
            h->matter_field = (double *)malloc(h->nsite * 10 * sizeof(double));
            if (!h->matter_field) return LBREF_ENOMEM;
        }
        memcpy(h->matter_field, M, h->nsite * (size_t)nc * sizeof(double));
        h->matter = 2;
    } else {
        memcpy(h->matter_uniform, M, (size_t)nc * sizeof(double));
        h->matter = 1;
    }
    h->matter_kind = kind;
    return LBREF_OK;
}

void lbref_lattice_d3q19(int *c, double *w) { (void)lbref_lattice(LBREF_D3Q19, c, w); }

int lbref_lattice(int lattice, int *c, double *w)
{
    if (lattice != LBREF_D3Q19 && lattice != LBREF_D2Q9) return LBREF_EINVAL;
    const int (*cq)[3] = lattice == LBREF_D2Q9 ? CQ9 : CQ19;
    const double *wq = lattice == LBREF_D2Q9 ? W9 : W19;
    for (int q = 0; q < lattice; ++q) {
        for (int m = 0; m < 3; ++m) c[q * 3 + m] = cq[q][m];
        w[q] = wq[q];
    }
    return lattice;
}

int lbref_lattice_q(const lbref *h) { return h ? h->nq : LBREF_EINVAL; }

int lbref_point_rhs(const double *in, int slicing, double *out)
{
    return lbref_point_rhs_matter(in, LBREF_MATTER_TENSOR, NULL, slicing, out);
}

int lbref_point_rhs_matter(const double *in, int kind, const double *M, int slicing, double *out)
{
    if (kind != LBREF_MATTER_TENSOR && kind != LBREF_MATTER_FLUID) return LBREF_EINVAL;
    if (!in || !out) return LBREF_EINVAL;
    const double alpha = in[0];
    double g6[6], K6[6], V[3], A[3], D[3][3][3], g[3][3], gi[3][3], K[3][3];
    double S6[6], Om[3], lam[3][6];
    for (int p = 0; p < 6; ++p) {
        g6[p] = in[1 + p];
        K6[p] = in[7 + p];
    }
    for (int k = 0; k < 3; ++k) {
        V[k] = in[13 + k];
        A[k] = in[16 + k];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[k][i][j] = in[19 + k * 6 + sym(i, j)];
    }
    full3(g6, g);
    full3(K6, K);
    inv3(g6, gi);
    double Q = 0.0;
    if (slicing == LBREF_SLICING_HARMONIC)
        Q = trace_up(gi, K);
    else if (slicing == LBREF_SLICING_ONE_PLUS_LOG)
        Q = trace_up(gi, K) / alpha;
    out[0] = -(alpha * alpha * Q);
    for (int p = 0; p < 6; ++p) out[1 + p] = -2.0 * alpha * K6[p];
    bm_sources(alpha, gi, g, K, V, A, D, kind, M, S6, Om);
    for (int p = 0; p < 6; ++p) out[7 + p] = alpha * S6[p];
    for (int k = 0; k < 3; ++k) out[13 + k] = Om[k];
    bm_lambda(gi, g, V, A, D, lam);
    for (int k = 0; k < 3; ++k)
        for (int p = 0; p < 6; ++p) out[16 + k * 6 + p] = lam[k][p];
    return LBREF_OK;
}

void lbref_point_feq(int kind, double u, const double *F, double *feq19)
{
    for (int q = 0; q < 19; ++q) {
        if (kind == 1) {
            double cF = 0.0;
            for (int m = 0; m < 3; ++m) cF += (double)CQ19[q][m] * F[m];
            feq19[q] = W19[q] * (u + 3.0 * cF);
        } else {
            feq19[q] = W19[q] * u;
        }
    }
}

int lbref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
