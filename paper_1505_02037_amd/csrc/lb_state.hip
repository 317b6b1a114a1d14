// lb_state.hip -- restoring distributions and checking the moments for
// non-finite values (checkpoint/resume and failure detection).
#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"
#include "lb_state.h"
#include "lb_step.h"

namespace lbnr {

// distributions at the current time (unpadded) back into the buffer, each at
// the position its pull reads (x - c_q): the inverse of the gather
template <class L>
__global__ void __launch_bounds__(256) k_scatter(const double *__restrict__ f, Geom G, double *__restrict__ fout)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    pull_sources(G, o);
#pragma unroll
    for (int F = 0; F < kFields; ++F)
#pragma unroll
        for (int q = 0; q < L::Q; ++q)
            plane<L>(fout, G, F, q)[o.src[q]] = f[((size_t)F * L::Q + q) * G.nsite + o.s];
}

// one field, FP32 deviations d = f - w u_rest
template <class L>
__global__ void __launch_bounds__(256) k_scatter32(const double *__restrict__ f, Geom G, int F,
                                                   float *__restrict__ fout)
{
    SiteT<L> o;
    if (!site_of(G, blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    pull_sources(G, o);
    const double ur = urest(F);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        plane<L>(fout, G, F, q)[o.src[q]] = (float)(f[(size_t)q * G.nsite + o.s] - L::w(q) * ur);
}

// a flag per block (any moment of its sites not finite), then one block ORs them
__global__ void __launch_bounds__(256) k_finite_partial(Geom G, const double *__restrict__ ubar,
                                                        int *__restrict__ flags)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (s < G.nsite) {
#pragma unroll
        for (int F = 0; F < kFields; ++F) {
            const double v = ubar[(size_t)F * G.ps + s];
            bad |= !(v - v == 0.0); // NaN and +-Inf give NaN
        }
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) flags[blockIdx.x] = bad;
}

__global__ void __launch_bounds__(256) k_finite_final(const int *__restrict__ flags, uint32_t nblocks,
                                                      int *__restrict__ out)
{
    int bad = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += blockDim.x) bad |= flags[b];
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) out[0] = bad;
}

static inline dim3 grid256(uint32_t n) { return dim3((n + 255) / 256); }

hipError_t launch_scatter(const double *f, const Geom &G, double *fout, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_scatter<D2Q9>, grid256(G.nsite), dim3(256), 0, st, f, G, fout);
    else
        hipLaunchKernelGGL(k_scatter<D3Q19>, grid256(G.nsite), dim3(256), 0, st, f, G, fout);
    return hipGetLastError();
}

hipError_t launch_scatter32(const double *f, const Geom &G, int field, float *fout, hipStream_t st)
{
    if (G.nq == D2Q9::Q)
        hipLaunchKernelGGL(k_scatter32<D2Q9>, grid256(G.nsite), dim3(256), 0, st, f, G, field, fout);
    else
        hipLaunchKernelGGL(k_scatter32<D3Q19>, grid256(G.nsite), dim3(256), 0, st, f, G, field, fout);
    return hipGetLastError();
}

size_t finite_scratch_ints(const Geom &G) { return (size_t)(G.nsite + 255) / 256 + 1; }

hipError_t launch_finite(const Geom &G, const double *ubar, int *scratch, hipStream_t st)
{
    const uint32_t nb = (G.nsite + 255) / 256;
    hipLaunchKernelGGL(k_finite_partial, dim3(nb), dim3(256), 0, st, G, ubar, scratch);
    hipLaunchKernelGGL(k_finite_final, dim3(1), dim3(256), 0, st, scratch, nb, scratch + nb);
    return hipGetLastError();
}

} // namespace lbnr
