// lb_state.h -- launchers of the state-transfer and check kernels
// (lb_state.hip): restoring distributions (the inverse of the gather) and the
// non-finite check of the moments.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "lb_kernels.h"

namespace lbnr {

// FP64 form: all fields' distributions at the current time ([16][Q][nsite])
// into the buffer, each at the position its pull reads.
hipError_t launch_scatter(const double *f, const Geom &G, double *fout, hipStream_t st);
// FP32-deviation form: one field's distributions ([Q][nsite], FP64) into the
// deviation buffer.
hipError_t launch_scatter32(const double *f, const Geom &G, int field, float *fout, hipStream_t st);

// ints of scratch launch_finite needs; the result is its last int
// (1: some moment is not finite)
size_t finite_scratch_ints(const Geom &G);
hipError_t launch_finite(const Geom &G, const double *ubar, int *scratch, hipStream_t st);

} // namespace lbnr
