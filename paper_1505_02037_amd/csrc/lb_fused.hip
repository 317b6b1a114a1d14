// lb_fused.hip -- the whole lattice Boltzmann step in one launch (z-marching).
//
// A workgroup of 256 threads owns a 14 x 14 column of sites and marches it
// through a chunk of up to 64 z-planes.  It collides a 16 x 16 tile per plane:
// its 14 x 14 sites plus a ring of one ghost site on every side, whose
// collisions are repeated redundantly so that every distribution arriving at
// an owned site is produced inside the workgroup.  That lets the launch also
// form the zeroth moments of the next step for its owned sites, through LDS,
// so a step reads every distribution once and writes it once:
//
//   per plane z of the chunk (plus one ghost plane below and above it)
//     1. corrected lapse/metric of plane z+1 on the 18 x 18 region around the
//        tile, from this step's moments, into a 3-plane LDS ring;
//     2. per thread: derivative stencil (in-plane neighbours from LDS, planes
//        z-1 and z+1 from the ring), sources, flux, then for each field: pull
//        its 19 distributions, relax them, store them if the site is owned,
//        and stage the 18 moving values in LDS;
//     3. owned threads gather what arrives at their column (the running sums
//        live in LDS): the in-plane
//        directions (for plane z), those moving up (for z+1) and those moving
//        down (for z-1), each summed in direction order; the moments of plane
//        z-1 are then complete: (in-plane + from below) + from above.
//
// The arithmetic per site is exactly that of the two-launch step (lb_step.h),
// so both paths return identical results.
#include <hip/hip_runtime.h>

#include "lb_device.h"
#include "lb_kernels.h"
#include "lb_site.h"
#include "lb_step.h"

namespace lbnr {

constexpr int kTile = 16;                 // collided tile edge
constexpr int kOwn = kTile - 2;           // owned interior edge
constexpr int kReg = kTile + 2;           // lapse/metric region edge
constexpr int kRegSites = kReg * kReg;    // 324
constexpr int kChunk = 64;                // z-planes per chunk
constexpr int kThreads = kTile * kTile;   // 256

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename T>
struct FusedShared {
    double lm[3][7][kRegSites];        // corrected lapse/metric, planes z-1, z, z+1
    T stage[kQ - 1][kThreads];         // post-collision values of the 18 moving directions
    double IB[kFields][kThreads];      // moments of plane z-1 so far: in-plane + from below
    double BL[kFields][kThreads];      // moments of plane z+1 so far: from below
};

// source position (in tile coordinates) of direction q for a site at (tx, ty)
__device__ __forceinline__ int src_slot(int q, int tx, int ty) { return (ty - cy(q)) * kTile + (tx - cx(q)); }

template <typename T, int Fld>
__device__ __forceinline__ void fused_field(const T *__restrict__ fin, T *__restrict__ fout, const Geom &G,
                                            const Site &o, const Params &P, double omega, double srcfac,
                                            bool store, bool owned_col, int tx, int ty, FusedShared<T> &sm,
                                            double *__restrict__ ubar_out, bool finish_prev, uint32_t s_prev)
{
    // the plane stride passes through an empty asm statement so that the
    // 304 plane addresses are formed per field instead of being kept live
    // across the z-loop
    size_t ps = G.ps;
    asm volatile("" : "+s"(ps));
    const T *fin_f = fin + (size_t)Fld * kQ * ps;
    T *fout_f = fout + (size_t)Fld * kQ * ps;
    T fl[kQ], out[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) fl[q] = fin_f[(size_t)q * ps + o.src[q]];
    if constexpr (sizeof(T) == 8)
        relax64<Fld>((const double *)fl, P, omega, srcfac, (double *)out);
    else
        relax32<Fld>((const float *)fl, P, (float)omega, srcfac, (float *)out);
    if (store) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) fout_f[(size_t)q * ps + o.s] = out[q];
    }
    const int t = ty * kTile + tx;
#pragma unroll
    for (int q = 1; q < kQ; ++q) sm.stage[q - 1][t] = out[q];
    __syncthreads();
    if (owned_col) {
        // what arrives at this column, grouped by the plane it comes from
        double in_plane = 0.0, below = 0.0, above = 0.0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const double v = (q == 0 || q == 5 || q == 6) ? (double)out[q]
                                                          : (double)sm.stage[q - 1][src_slot(q, tx, ty)];
            if (cz(q) == 0)
                in_plane += v;   // arrives in plane z
            else if (cz(q) > 0)
                below += v;      // arrives in plane z+1, from below
            else
                above += v;      // arrives in plane z-1, from above
        }
        if (finish_prev) {
            double u = sm.IB[Fld][t] + above;
            if constexpr (sizeof(T) == 4) u = urest(Fld) + u;
            ubar_out[(size_t)Fld * ps + s_prev] = u;
        }
        sm.IB[Fld][t] = in_plane + sm.BL[Fld][t];
        sm.BL[Fld][t] = below;
    }
    __syncthreads(); // staged values read before the next field overwrites them
    if constexpr (Fld + 1 < kFields)
        fused_field<T, Fld + 1>(fin, fout, G, o, P, omega, srcfac, store, owned_col, tx, ty, sm, ubar_out,
                                finish_prev, s_prev);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fused(const T *__restrict__ fin, T *__restrict__ fout, Geom G,
                                                    int slicing, double omega, double srcfac,
                                                    const double *__restrict__ ubar_in,
                                                    double *__restrict__ ubar_out, int ntx, int nty, int ntz)
{
    __shared__ FusedShared<T> sm;
    // XCD-aware order: consecutive workgroups land on different XCDs, so give
    // each XCD a contiguous range of tiles (neighbours share ghost reads in L2)
    const int ntiles = ntx * nty * ntz;
    const int per = (ntiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= ntiles) return;
    const int bx = tile % ntx, by = (tile / ntx) % nty, bz = tile / (ntx * nty);

    const int t = threadIdx.x, tx = t % kTile, ty = t / kTile;
    const int ox = bx * kOwn - 1, oy = by * kOwn - 1; // tile origin (unwrapped)
    const int z0 = bz * kChunk;
    const int z1 = z0 + kChunk < G.nz ? z0 + kChunk : G.nz;
    const int gx = ox + tx, gy = oy + ty;
    const int wx = wrapi(gx, G.nx), wy = wrapi(gy, G.ny);
    const bool owned_col = tx >= 1 && tx <= kOwn && ty >= 1 && ty <= kOwn && gx < G.nx && gy < G.ny;

    // corrected lapse/metric of plane p on the region around the tile
    auto region_lm = [&](int p) {
        const int slot = wrapi(p - (z0 - 2), 3);
        const int zz = wrapi(p, G.nz);
        for (int r = t; r < kRegSites; r += kThreads) {
            const int rx = wrapi(ox - 1 + r % kReg, G.nx), ry = wrapi(oy - 1 + r / kReg, G.ny);
            const uint32_t s = ((uint32_t)zz * (uint32_t)G.ny + (uint32_t)ry) * (uint32_t)G.nx + (uint32_t)rx;
            double ub[13], c[7], R[7];
#pragma unroll
            for (int F = 0; F < 13; ++F) ub[F] = ubar_in[(size_t)F * G.ps + s];
            lapse_metric(ub, slicing, c, R);
#pragma unroll
            for (int k = 0; k < 7; ++k) sm.lm[slot][k][r] = c[k];
        }
    };
    auto own_moments = [&](int p, double ub[kFields]) {
        const uint32_t s =
            ((uint32_t)wrapi(p, G.nz) * (uint32_t)G.ny + (uint32_t)wy) * (uint32_t)G.nx + (uint32_t)wx;
#pragma unroll
        for (int F = 0; F < kFields; ++F) ub[F] = ubar_in[(size_t)F * G.ps + s];
    };

    double ub[kFields];
#pragma unroll
    for (int F = 0; F < kFields; ++F) sm.IB[F][t] = sm.BL[F][t] = 0.0;
    region_lm(z0 - 2);
    region_lm(z0 - 1);
    own_moments(z0 - 1, ub);

    const int rc = (ty + 1) * kReg + (tx + 1); // own site in region coordinates
    for (int z = z0 - 1; z <= z1; ++z) {
        region_lm(z + 1);
        __syncthreads();
        // stencil at plane z from the region ring (same arithmetic as stencil())
        const int sm1 = wrapi(z - 1 - (z0 - 2), 3), s0 = wrapi(z - (z0 - 2), 3), sp1 = wrapi(z + 1 - (z0 - 2), 3);
        double c[7], Rag[7], A[3], D[18];
        lapse_metric(ub, slicing, c, Rag);
        {
            const int np[3] = {rc + 1, rc + kReg, rc};
            const int nm[3] = {rc - 1, rc - kReg, rc};
            const int slp[3] = {s0, s0, sp1};
            const int slm[3] = {s0, s0, sm1};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = (sm.lm[slp[k]][0][np[k]] - sm.lm[slm[k]][0][nm[k]]) / (2.0 * c[0]);
#pragma unroll
                for (int p = 0; p < 6; ++p) D[k * 6 + p] = (sm.lm[slp[k]][1 + p][np[k]] - sm.lm[slm[k]][1 + p][nm[k]]) * 0.25;
            }
        }
        Params P;
        params_from(ub, c, Rag, A, D, P);
        Site o;
        o.x = wx;
        o.y = wy;
        o.z = wrapi(z, G.nz);
        o.s = ((uint32_t)o.z * (uint32_t)G.ny + (uint32_t)wy) * (uint32_t)G.nx + (uint32_t)wx;
        pull_sources(G, o);
        const bool store = owned_col && z >= z0 && z < z1;
        const bool finish_prev = z - 1 >= z0 && z - 1 < z1;
        const uint32_t s_prev =
            ((uint32_t)wrapi(z - 1, G.nz) * (uint32_t)G.ny + (uint32_t)wy) * (uint32_t)G.nx + (uint32_t)wx;
        fused_field<T, 0>(fin, fout, G, o, P, omega, srcfac, store, owned_col, tx, ty, sm, ubar_out, finish_prev,
                          s_prev);
        if (z < z1) own_moments(z + 1, ub);
    }
}

void fused_grid(const Geom &G, int *ntx, int *nty, int *ntz, int *blocks)
{
    *ntx = (G.nx + kOwn - 1) / kOwn;
    *nty = (G.ny + kOwn - 1) / kOwn;
    *ntz = (G.nz + kChunk - 1) / kChunk;
    const int ntiles = *ntx * *nty * *ntz;
    *blocks = 8 * ((ntiles + 7) / 8);
}

hipError_t launch_fused64(const double *fin, double *fout, const Geom &G, int slicing, double omega, double srcfac,
                          const double *ubar_in, double *ubar_out, hipStream_t st)
{
    int ntx, nty, ntz, blocks;
    fused_grid(G, &ntx, &nty, &ntz, &blocks);
    hipLaunchKernelGGL(k_fused<double>, dim3(blocks), dim3(kThreads), 0, st, fin, fout, G, slicing, omega, srcfac,
                       ubar_in, ubar_out, ntx, nty, ntz);
    return hipGetLastError();
}

hipError_t launch_fused32(const float *fin, float *fout, const Geom &G, int slicing, double omega, double srcfac,
                          const double *ubar_in, double *ubar_out, hipStream_t st)
{
    int ntx, nty, ntz, blocks;
    fused_grid(G, &ntx, &nty, &ntz, &blocks);
    hipLaunchKernelGGL(k_fused<float>, dim3(blocks), dim3(kThreads), 0, st, fin, fout, G, slicing, omega, srcfac,
                       ubar_in, ubar_out, ntx, nty, ntz);
    return hipGetLastError();
}

} // namespace lbnr
