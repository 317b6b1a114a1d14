// lb_kernels.h -- host-callable launchers of the device kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbnr {

// Slicing codes (section "Gauge choices"): Q = tr K (harmonic), Q = 0
// (geodesic), Q = tr K / alpha ("1+log").
constexpr int kSlicingHarmonic = 0;
constexpr int kSlicingGeodesic = 1;
constexpr int kSlicingOnePlusLog = 2;

// Matter kinds: the tensor G^00, G^0_k, G_ij (10 values), or a perfect fluid
// (rho, P) at rest in the slicing.
constexpr int kMatterTensor = 0;
constexpr int kMatterFluid = 1;

// Collision: BGK (Eq. numlb) or the declared regularized variant (the
// non-equilibrium part keeps only its zeroth and first moments).
constexpr int kCollisionBgk = 0;
constexpr int kCollisionRegularized = 1;

// Lattice geometry as the kernels see it.
struct Geom {
    int nx, ny, nz;
    uint32_t nsite;  // nx * ny * nz
    size_t ps;       // plane stride in elements (nsite rounded up to 64)
    int nq = 19;     // directions of the lattice: 19 (D3Q19) or 9 (D2Q9, nz = 1)
};

// Matter in the sources, as the kernels take it: the values of one kind
// (10 for the tensor kind, 2 for the fluid kind) either per site, from
// `field` ([ncomp][ps]), or the same at every site, from `uni` (carried in the
// kernel arguments).  kind < 0: vacuum.
struct MatterArg {
    const double *field = nullptr;
    int kind = -1;
    double uni[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
};

// FP64 form (lb_fp64.hip); the split-step launchers, the initialisation and
// the gather run the lattice G.nq names
hipError_t launch_moments(const double *fin, const Geom &G, int slicing, double *ubar, double *lm, hipStream_t st);
hipError_t launch_collide(const double *fin, double *fout, const Geom &G, int slicing, double omega,
                          double srcfac, const double *ubar, const double *lm, const MatterArg &m, int collision,
                          hipStream_t st);
hipError_t launch_output(const Geom &G, int slicing, const double *ubar, const double *lm, double *u,
                         const MatterArg &m, hipStream_t st);
hipError_t launch_init(const Geom &G, int slicing, const double *u0, double *lm, double *fout, const MatterArg &m,
                       hipStream_t st);
hipError_t launch_gather(const double *fin, const Geom &G, double *f, hipStream_t st);
hipError_t launch_copy_lm(const Geom &G, const double *u0, double *lm, hipStream_t st);
size_t norm_scratch_doubles(const Geom &G);
hipError_t launch_norms(const Geom &G, const double *u, const double *ref, double *scratch, hipStream_t st);

// FP32-deviation form (lb_fp32.hip); the output and norm kernels are shared
hipError_t launch_moments32(const float *fin, const Geom &G, int slicing, double *ubar, double *lm, hipStream_t st);
hipError_t launch_collide32(const float *fin, float *fout, const Geom &G, int slicing, double omega, double srcfac,
                            const double *ubar, const double *lm, const MatterArg &m, int collision,
                            hipStream_t st);
hipError_t launch_init32(const Geom &G, int slicing, const double *u0, double *lm, float *fout, const MatterArg &m,
                         hipStream_t st);
hipError_t launch_gather32(const float *fin, const Geom &G, int field, double *f, hipStream_t st);

// one-launch z-marching step (lb_fused.hip): reads this step's moments
// ubar_in, writes the post-collision distributions and the next step's
// moments ubar_out
hipError_t launch_fused64(const double *fin, double *fout, const Geom &G, int slicing, double omega, double srcfac,
                          const double *ubar_in, double *ubar_out, hipStream_t st);
hipError_t launch_fused32(const float *fin, float *fout, const Geom &G, int slicing, double omega, double srcfac,
                          const double *ubar_in, double *ubar_out, hipStream_t st);

} // namespace lbnr
