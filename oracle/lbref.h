/*
 * lbref.h -- FP64 CPU oracle of the lattice Boltzmann step for the Bona-Masso
 * flux-conservative Einstein system (Ilseven & Mendoza, "Lattice Boltzmann
 * Model for Numerical Relativity").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Conventions (lattice units dt = dx = 1):
 *   fields (16):  0 alpha | 1..6 gamma_ij | 7..12 K_ij | 13..15 V_k,
 *                 symmetric pairs in the order xx, xy, xz, yy, yz, zz.
 *   u arrays:     u[field][z][y][x], x fastest, float64.
 *   f arrays:     f[field][q][z][y][x], the distributions at the current time
 *                 (after streaming), directions q in the paper's order of the
 *                 lattice (D3Q19, or D2Q9 on an nx x ny x 1 lattice).
 *   boundaries:   periodic in all three directions (section "Gauge choices").
 *
 * Return codes: 0 on success, negative on error (see LBREF_E*).
 */
#ifndef LBREF_H
#define LBREF_H

#ifdef __cplusplus
extern "C" {
#endif

#define LBREF_OK 0
#define LBREF_EINVAL (-1)
#define LBREF_ENOMEM (-2)

#define LBREF_D3Q19 19 /* section "Lattice Boltzmann Model", D3Q19 matrix */
#define LBREF_D2Q9 9   /* section "Lattice Boltzmann Model", D2Q9 matrix; nz = 1 */

#define LBREF_SLICING_HARMONIC 0 /* Q = tr K   (section "Gauge choices") */
#define LBREF_SLICING_GEODESIC 1 /* Q = 0 */
#define LBREF_SLICING_ONE_PLUS_LOG 2 /* Q = tr K / alpha ("1+log") */

typedef struct lbref lbref;

/* nx, ny, nz >= 1; tau > 1/2 (relaxation time in units of dt).  D3Q19. */
int lbref_create(int nx, int ny, int nz, double tau, int slicing, lbref **out);
/* The same on a chosen lattice: LBREF_D3Q19, or LBREF_D2Q9 (requires nz = 1). */
int lbref_create_lattice(int lattice, int nx, int ny, int nz, double tau, int slicing, lbref **out);
/* number of directions of the handle's lattice */
int lbref_lattice_q(const lbref *h);
void lbref_destroy(lbref *h);

/* Initial distributions from macroscopic fields u0 (16 x nsite):
 * f_q = f^eq_q(u0) - w_q R(u0)/2, every quantity evaluated at u0. */
int lbref_init_fields(lbref *h, const double *u0);

/* Advance nsteps lattice Boltzmann steps. */
int lbref_step(lbref *h, long long nsteps);

/* Macroscopic fields u = sum_q f_q + R/2 at the current time (16 x nsite). */
int lbref_moments(lbref *h, double *u_out);

/* Copy the current distributions out / in (16 x Q x nsite). */
int lbref_get_distributions(const lbref *h, double *f_out);
int lbref_set_distributions(lbref *h, const double *f_in);

long long lbref_nsteps_done(const lbref *h);

/* Collision: LBREF_COLLISION_BGK (Eq. numlb, the default) or the declared
 * variant LBREF_COLLISION_REGULARIZED, which keeps of the non-equilibrium part
 * f - f^eq only its zeroth and first moments (relaxed as BGK relaxes them):
 *   f* = f^eq + (1 - omega) w_q (m0 + c_q.J / c_s^2) + w_q (1 - omega/2) R,
 *   m0 = sum_q (f - f^eq),  J = sum_q c_q (f - f^eq).
 * The paper suggests a stabilised collision (an entropic one) without
 * specifying it; this variant is not the paper's method. */
#define LBREF_COLLISION_BGK 0
#define LBREF_COLLISION_REGULARIZED 1
int lbref_set_collision(lbref *h, int kind);

/* Matter (energy-momentum tensor G, units c = 8 pi G = 1; section
 * "Bona-Masso evolution equations"), in lattice units, of one of two kinds:
 *   LBREF_MATTER_TENSOR: 10 values, G^00, G^0_k (x, y, z), G_ij (xx, xy, xz,
 *                        yy, yz, zz);
 *   LBREF_MATTER_FLUID:  2 values, rho and P of a perfect fluid at rest in
 *                        the slicing: G^00 = rho / alpha^2, G^0_k = 0,
 *                        G_ij = P gamma_ij at the site's lapse and metric
 *                        (section "Expansion of flat universe").
 * per_site = 0: M holds the values used at every site; 1: M is
 * [ncomp][nsite].  M = NULL returns to vacuum.  The matter set enters every
 * later evaluation of the sources (initialisation, steps, moments) until it
 * is changed. */
#define LBREF_MATTER_TENSOR 0
#define LBREF_MATTER_FLUID 1
int lbref_set_matter(lbref *h, int kind, const double *M, int per_site);

/* ---- point routines, exposed so tests can pin the formulas ---- */

/* D3Q19 velocities c[q*3+m] and weights w[q]. */
void lbref_lattice_d3q19(int *c, double *w);
/* velocities and weights of a lattice (c: 3 Q ints, w: Q doubles); returns Q */
int lbref_lattice(int lattice, int *c, double *w);

/* Right-hand sides and flux of the Bona-Masso system at one point.
 * in  (37): alpha, gamma[6], K[6], V[3], A[3], D[18] with D[k*6+pair] = D_k(ij)
 * out (34): R_alpha, R_gamma[6], R_K[6] (= alpha S_ij), Omega[3],
 *           lambda[18] with lambda[k*6+pair] = lambda^k_(ij) */
int lbref_point_rhs(const double *in, int slicing, double *out);
/* The same with matter M of the given kind (as for lbref_set_matter; NULL:
 * vacuum). */
int lbref_point_rhs_matter(const double *in, int kind, const double *M, int slicing, double *out);

/* Equilibrium of one field at one point on D3Q19: kind 0 -> w_q u (alpha, gamma, V);
 * kind 1 -> w_q (u + c_q.F / c_s^2) (K components), F = flux vector (3). */
void lbref_point_feq(int kind, double u, const double *F, double *feq19);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int lbref_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
