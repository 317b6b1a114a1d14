/*
 * lb.h -- C-ABI of the MI355X (gfx950) lattice Boltzmann step for the
 * Bona-Masso flux-conservative Einstein system (Ilseven & Mendoza,
 * "Lattice Boltzmann Model for Numerical Relativity").
 *
 * The library evolves the 16 fields u = (alpha, gamma_ij, K_ij, V_k) of the
 * Bona-Masso system (section "Bona-Masso evolution equations", vacuum, zero
 * shift) with one distribution per field on the D3Q19 velocity set, or on
 * D2Q9 for lattices one site thick in z (section "Lattice Boltzmann Model"),
 * BGK collision with a source term (Eq. numlb),
 * the per-field equilibria and sources (Eqs. alfa .. ekstsor) and the
 * half-source macroscopic moments, on a periodic lattice (section "Gauge
 * choices").  Lattice units: dt = dx = 1.
 *
 * Conventions shared by every entry point
 *   fields   0 alpha | 1..6 gamma (xx,xy,xz,yy,yz,zz) | 7..12 K (same order)
 *            | 13..15 V (x,y,z)
 *   u arrays double, [16][nz][ny][nx], x fastest, no padding.
 *   f arrays double, [16][Q][nz][ny][nx], the distributions at the current
 *            time after streaming, the lattice's Q directions in the paper's
 *            order.
 *   pointers "on_device" = 1: a device pointer on the handle's device (the
 *            call is stream-ordered on the handle's stream, which does not
 *            wait for other streams: device inputs must be complete when the
 *            call is made); 0: host memory (the call copies synchronously).
 *            The caller owns every array it passes; the library copies what
 *            it needs and keeps no pointer.
 *   errors   every int-returning function returns LB_OK (0) or a negative
 *            LB_E* code; lb_strerror names it.  A failed call leaves the
 *            handle usable unless it returns LB_EDEVICE.
 *   threads  one handle is driven from one host thread at a time.
 */
#ifndef LBNR_LB_H
#define LBNR_LB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)    /* bad argument or configuration */
#define LB_ENOMEM (-2)    /* device or host allocation failed */
#define LB_EDEVICE (-3)   /* a HIP call failed (message in lb_last_error) */
#define LB_ESTATE (-4)    /* handle not initialised with lb_init_fields */

#define LB_D3Q19 19 /* section "Lattice Boltzmann Model", D3Q19 matrix */
#define LB_D2Q9 9    /* section "Lattice Boltzmann Model", D2Q9 matrix: the
                        paper's gauge-wave lattice; requires nz = 1 and the
                        split path (LB_PATH_AUTO or LB_PATH_SPLIT) */

#define LB_SLICING_HARMONIC 0 /* Q = tr K  (harmonic slicing)  */
#define LB_SLICING_GEODESIC 1 /* Q = 0     (geodesic slicing)  */
#define LB_SLICING_ONE_PLUS_LOG 2 /* Q = tr K / alpha ("1+log" slicing; the
                                     paper names it in section "Gauge
                                     choices" and evaluates only the other
                                     two: a declared variant) */

#define LB_FP64 0      /* distributions stored and collided in FP64 */
#define LB_FP32_DEV 1  /* distributions stored and streamed in FP32 as
                          deviations from the rest-state equilibrium
                          (alpha = 1, gamma = delta, K = V = 0), relaxed in
                          FP32; moments, the lapse/metric correction, the
                          derivative stencil, the geometry, the sources, the
                          flux and the error norms stay FP64 */

#define LB_PATH_AUTO 0   /* the faster of the two on MI355X: split */
#define LB_PATH_SPLIT 1  /* two launches per step: moments, then collide */
#define LB_PATH_FUSED 2  /* one z-marching launch per step that also forms
                            the next step's moments (same results) */

#define LB_COLLISION_BGK 0          /* BGK with source (Eq. numlb) */
#define LB_COLLISION_REGULARIZED 1  /* declared variant, not the paper's: of
                                       the non-equilibrium part f - f^eq only
                                       its zeroth and first moments are kept
                                       and relaxed as BGK relaxes them,
                                       f* = f^eq + (1 - 1/tau) w (m0 + c.J/c_s^2)
                                          + w (1 - 1/(2 tau)) R;
                                       same moments and first-order dynamics,
                                       no higher non-equilibrium moments (the
                                       paper suggests a stabilised collision
                                       without specifying one).  It delays
                                       the blow-up for tau <= 0.65 and ends
                                       runs earlier for tau >= 1.5; split
                                       path only */

typedef struct lb_handle lb_handle; /* opaque, owned by the library */

/* Optional device allocator for the memory a handle holds (distribution
 * buffers, per-site scratch, per-site matter): dev_alloc(bytes, ctx) returns
 * `bytes` of device memory on the handle's device (the device is current
 * during the call), aligned to at least 256 bytes, or NULL if it has none;
 * dev_free(ptr, ctx) gives back what dev_alloc returned.  The library calls
 * dev_free only after the handle's stream has finished with the memory.
 * Lets a caller serve the library from its own pool (for example a
 * framework's caching allocator). */
typedef void *(*lb_dev_alloc_fn)(size_t bytes, void *ctx);
typedef void (*lb_dev_free_fn)(void *ptr, void *ctx);

typedef struct lb_config {
    int lattice;     /* LB_D3Q19 or LB_D2Q9 */
    int nx, ny, nz;  /* periodic extents, each >= 1 */
    double tau;      /* relaxation time in units of dt (Eq. lbe); > 1/2 */
    int slicing;     /* LB_SLICING_HARMONIC, LB_SLICING_GEODESIC or
                        LB_SLICING_ONE_PLUS_LOG */
    int precision;   /* LB_FP64 or LB_FP32_DEV */
    int device;      /* HIP device ordinal, or -1 for the current device */
    void *stream;    /* hipStream_t to run on, or NULL: the library creates
                        and owns a stream of default priority */
    int path;        /* LB_PATH_AUTO, LB_PATH_SPLIT or LB_PATH_FUSED: how a
                        step is launched; every path gives identical results */
    int collision;   /* LB_COLLISION_BGK (0) or LB_COLLISION_REGULARIZED */
    lb_dev_alloc_fn dev_alloc; /* NULL: the library uses hipMalloc/hipFree */
    lb_dev_free_fn dev_free;   /* required with dev_alloc */
    void *alloc_ctx;           /* passed to dev_alloc and dev_free */
} lb_config;

/* Allocates two distribution buffers and per-site scratch on the device
 * (through cfg->dev_alloc if set).  Fails with LB_EINVAL on a bad config
 * (dev_alloc without dev_free included), LB_ENOMEM if the device memory is
 * not available (or dev_alloc returns NULL).  *out is set to NULL on
 * failure, with everything allocated so far given back. */
int lb_create(const lb_config *cfg, lb_handle **out);

/* Device bytes lb_create would allocate for cfg (0 on a bad config). */
size_t lb_device_bytes(const lb_config *cfg);

/* Initial distributions from the fields u0 ([16][nz][ny][nx]):
 * f_q = f^eq_q(u0) - w_q R(u0)/2 with every quantity (right-hand sides R,
 * derivatives of the lapse and metric, flux) evaluated at u0, so that the
 * half-source moments at t = 0 return u0 up to O(dt^2).  The paper leaves the
 * initial distributions open; this is the equilibrium of its Eqs. alfa ..
 * ekst shifted by the half source of its moment definition.  Resets the step
 * counter.  Synchronises the handle's stream, so u0 may be released on
 * return. */
int lb_init_fields(lb_handle *h, const double *u0, int on_device);

/* Enqueues nsteps time steps on the handle's stream; does not synchronise.
 * One step (Eq. numlb): pull streaming, moments with half source, the lapse
 * and metric corrected first and differentiated (paragraph after the
 * first-order derivative definitions), the sources (extrinsic-curvature and
 * momentum-variable equations, Eq. Vsor) and flux, and BGK relaxation towards
 * the equilibria with the source added (Eqs. alfa .. ekstsor).  nsteps >= 0
 * (LB_EINVAL otherwise); LB_ESTATE before lb_init_fields or
 * lb_set_distributions. */
int lb_step(lb_handle *h, long long nsteps);

/* Macroscopic fields u = sum_q f_q + R/2 at the current time into u_out
 * ([16][nz][ny][nx]): the moments with half the source (section "Lattice
 * Boltzmann Model").  Synchronises the handle's stream.  LB_ESTATE before
 * the state is set. */
int lb_moments(lb_handle *h, double *u_out, int on_device);

/* The distributions at the current time into f_out ([16][Q][nz][ny][nx],
 * Q = 19 on D3Q19, 9 on D2Q9, directions in the paper's order).
 * Synchronises the handle's stream. */
int lb_get_distributions(lb_handle *h, double *f_out, int on_device);

/* Checkpoint/resume: replaces the state by the distributions f_in
 * ([16][Q][nz][ny][nx], the layout lb_get_distributions writes), the exact
 * inverse of lb_get_distributions in the FP64 form (resuming from a saved
 * state continues bit for bit; saving only the fields u and calling
 * lb_init_fields would drop the non-equilibrium part).  In the FP32-deviation
 * form the values are rounded to FP32 deviations again.  Resets the step
 * counter; the handle counts as initialised.  Synchronises the handle's
 * stream, so f_in may be released on return. */
int lb_set_distributions(lb_handle *h, const double *f_in, int on_device);

/* Failure check: *all_finite = 1 if every moment of every site is finite,
 * 0 if any is NaN or infinite (the scheme's blow-up); computed on the device
 * (one moments pass and a reduction).  Synchronises the handle's stream. */
int lb_check_finite(lb_handle *h, int *all_finite);

/* Matter: the energy-momentum tensor G (units c = 8 pi G = 1, lattice units)
 * in the sources of the extrinsic-curvature and momentum-variable equations
 * (section "Bona-Masso evolution equations"; section "Expansion of flat
 * universe" for the fluid).  Two kinds:
 *   LB_MATTER_TENSOR  10 values: G^00, G^0_k (x, y, z), G_ij (xx, xy, xz, yy,
 *                     yz, zz);
 *   LB_MATTER_FLUID    2 values: rho and P of a perfect fluid at rest in the
 *                     slicing; alpha^2 G^00 = rho, G^0_k = 0, G_ij = P gamma_ij
 *                     at each site's lapse and metric.
 * per_site = 0: M holds the values for every site; 1: M is [ncomp][nz][ny][nx].
 * M = NULL returns to vacuum.  The matter set enters every later call that
 * evaluates the sources (lb_init_fields, lb_step, lb_moments, lb_error_norms)
 * until it is changed; values for every site are carried in the launch
 * arguments, values per site are copied to the device (stream-ordered after
 * the steps already enqueued).  A time-dependent matter field is followed by
 * setting it before each step (the step from time n uses the matter of time
 * n) and before each read-out.  LB_EINVAL on an unknown kind, or on a handle
 * of the fused path (its launch evaluates vacuum sources only). */
#define LB_MATTER_TENSOR 0
#define LB_MATTER_FLUID 1
int lb_set_matter(lb_handle *h, int kind, const double *M, int per_site, int on_device);

/* Error norms of the current fields against u_ref ([16][nz][ny][nx]),
 * computed on the device in FP64 (the error measures of section "Analysis
 * and Simulation Errors" are formed from these).  Per field F (arrays of 16):
 *   max_abs[F] = max_x |u_F - ref_F|,  l2[F] = sqrt(sum_x (u_F - ref_F)^2 / N),
 *   ref_max[F] = max_x |ref_F|.
 * Any output pointer may be NULL.  Synchronises the handle's stream. */
int lb_error_norms(lb_handle *h, const double *u_ref, int on_device,
                   double *max_abs, double *l2, double *ref_max);

/* Steps taken since lb_init_fields. */
long long lb_steps_done(const lb_handle *h);

/* Enables (1) or disables (0) HIP-event timing of the step kernels.  A timed
 * lb_step records an event around every launch and synchronises the stream
 * after every 256 steps and at its end. */
int lb_set_timing(lb_handle *h, int enable);

/* Average device time in milliseconds of each kernel of the last lb_step
 * call that ran with timing enabled, measured with HIP events on the
 * handle's stream.  names[i] (static strings: the kernels' template-instance
 * names as a profiler lists them, e.g. "lbnr::k_collide<lbnr::D3Q19, false,
 * 0>" for lattice, matter, collision) and ms[i] for i < *count (at most cap
 * entries).  Returns LB_ESTATE if no timed call has run. */
int lb_kernel_times(lb_handle *h, const char **names, double *ms, int cap, int *count);

/* Waits for the handle's stream, frees its device memory (through the
 * config's dev_free if it named an allocator) and its stream if the library
 * created it.  NULL is ignored. */
void lb_destroy(lb_handle *h);

/* Static text naming an LB_* code. */
const char *lb_strerror(int code);
/* Text of the last HIP failure seen by this thread in any lb_* or lb_server_*
 * call (empty if none; a later successful call does not clear it). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBNR_LB_H */
