/*
 * hbm_probe.h -- plain device-to-device copies and reads of known size.
 *
 * Not part of the lattice Boltzmann method: it measures the card's achievable
 * HBM bandwidth (a copy reads and writes every byte once), calibrates the
 * HBM traffic counters (FETCH_SIZE / WRITE_SIZE of a copy of B bytes each
 * way), and tells whether a re-read of recently read data is served faster
 * (by the Infinity Cache) than a first read.  The roofline figures of the
 * method's kernels are quoted against the vendor peak and against these
 * measured ceilings.
 */
#ifndef LBNR_HBM_PROBE_H
#define LBNR_HBM_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Allocates two device buffers of `bytes` each (bytes a multiple of 64) on
 * the current device, copies src -> dst `reps` times with a streaming copy
 * kernel (16-byte loads and stores), and returns the average milliseconds per
 * copy in *ms (HIP events).  Returns 0, or -1 on a bad argument, -2 if the
 * allocation fails, -3 on any other HIP error.  Frees what it allocated. */
int hbm_copy_probe(size_t bytes, int reps, double *ms);

/* Same, for a read-only stream over one buffer of `bytes` (the result of the
 * reduction is kept on the device); *ms is the average per pass. */
int hbm_read_probe(size_t bytes, int reps, double *ms);

/* Re-read test: reads a buffer of `bytes` and times an immediate second read
 * (*ms_hot); reads it, then a separate buffer of `flush_bytes`, and times a
 * read of the first buffer again (*ms_cold).  Best of `reps` of each, in
 * milliseconds.  bytes and flush_bytes multiples of 64; return codes as for
 * hbm_copy_probe. */
int hbm_reread_probe(size_t bytes, size_t flush_bytes, int reps, double *ms_hot, double *ms_cold);

#ifdef __cplusplus
}
#endif
#endif
