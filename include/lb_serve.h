/*
 * lb_serve.h -- continuous batching of independent lattice Boltzmann
 * evolutions on one GPU (C-ABI).
 *
 * Requests are independent periodic evolutions of the Bona-Masso system (the
 * step of include/lb.h: same arithmetic, same results bit for bit) with their
 * own lattice size, relaxation time, slicing, initial fields and step count.
 * The server keeps every admitted request's distributions resident in one
 * device arena sized by an HBM budget and advances all resident requests
 * together: each time step is two batched launches over a work list of
 * (request, 256-site block) items plus a small bookkeeping launch, and
 * `steps_per_launch` such steps are replayed as one captured HIP graph.  Each
 * request stops at exactly its own step count inside a graph (its counter
 * lives on the device).  Between graph launches the host admits queued
 * requests that fit (arrival order, any request that fits may pass one that
 * does not) and retires finished ones, so requests that arrive while others
 * run join them as memory and slots free up.
 *
 * Conventions as in include/lb.h (u arrays are host double [16][nz][ny][nx]).
 * Every int-returning function returns LB_OK or a negative LB_E* code; after
 * LB_EDEVICE, lb_last_error() names the failed HIP call.  A device that cannot
 * be made current is LB_EDEVICE.  One server is driven from one host thread at
 * a time.
 */
#ifndef LBNR_LB_SERVE_H
#define LBNR_LB_SERVE_H

#include <stddef.h>

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LB_REQ_QUEUED 0   /* submitted, waiting for memory or a slot */
#define LB_REQ_RUNNING 1  /* resident on the device */
#define LB_REQ_DONE 2     /* finished, result available */
#define LB_REQ_FAILED 3   /* finished, but its fields are not finite */

typedef struct lb_server lb_server; /* opaque */

typedef struct lb_server_config {
    size_t hbm_budget_bytes; /* device arena shared by the resident requests */
    int precision;           /* LB_FP64 or LB_FP32_DEV, for every request */
    int max_resident;        /* slot limit (>= 1) */
    int steps_per_launch;    /* time steps per graph launch (>= 1) */
    int device;              /* HIP device ordinal or -1 (current) */
    void *stream;            /* hipStream_t or NULL (the server owns one) */
} lb_server_config;

typedef struct lb_request_info {
    int state;                  /* LB_REQ_* */
    long long steps_done;       /* steps applied so far */
    double t_submit;            /* host monotonic seconds at lb_server_submit */
    double t_admit;             /* ... when it became resident (0 if not yet) */
    double t_done;              /* ... when its result was copied out (0 if not) */
} lb_request_info;

typedef struct lb_server_stats {
    long long graph_launches;
    long long site_updates;     /* sum over requests of sites x steps applied */
    long long completed;
    long long failed;
    int resident;
    int queued;
    size_t arena_bytes;         /* size of the device arena */
    size_t arena_in_use;        /* bytes held by resident requests now */
    size_t arena_peak;          /* most bytes ever held at once */
} lb_server_stats;

/* Allocates the arena (hbm_budget_bytes) on the device.  LB_ENOMEM if it does
 * not fit, LB_EINVAL on a bad config. */
int lb_server_create(const lb_server_config *cfg, lb_server **out);

/* Device bytes one request of this lattice needs inside the arena. */
size_t lb_server_request_bytes(const lb_server *s, const lb_config *cfg);

/* Queues an evolution of nsteps >= 0 steps from u0 (host, copied).  cfg's
 * lattice (LB_D3Q19 only), extents, tau and slicing are used; its precision,
 * device, stream and allocator are ignored (the server's apply; requests
 * live in the server's arena).  LB_EINVAL if cfg is
 * invalid, names another lattice, or the request can never fit the arena.
 * *id receives the request id. */
int lb_server_submit(lb_server *s, const lb_config *cfg, const double *u0, long long nsteps,
                     unsigned long long *id);

/* One scheduling round: admit what fits, run one graph launch of
 * steps_per_launch steps over the resident requests (skipped if none),
 * wait for it, and copy out the results of requests that finished.
 * *active (may be NULL) receives resident + queued requests afterwards. */
int lb_server_advance(lb_server *s, int *active);

int lb_server_info(const lb_server *s, unsigned long long id, lb_request_info *info);

/* Copies the finished request's fields u = sum f + R/2 to u_out (host) and
 * forgets the request.  LB_ESTATE if it has not finished. */
int lb_server_result(lb_server *s, unsigned long long id, double *u_out);

int lb_server_get_stats(const lb_server *s, lb_server_stats *st);

void lb_server_destroy(lb_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LBNR_LB_SERVE_H */
