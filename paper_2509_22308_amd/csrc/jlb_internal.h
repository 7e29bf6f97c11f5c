// Internal interface between the host driver (jlb_host.cpp) and the gfx950
// kernels (jlb_device.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jlb {

// Material id in the low two bits of a mask byte.
enum : uint8_t { MAT_VACUUM = 0, MAT_REGION2 = 1, MAT_REGION3 = 2, MAT_PEC = 3 };
// Conductor-neighbour bits: the neighbour a population is pulled from is a
// perfect conductor.  Named by the population that is affected.
enum : uint8_t {
    NB_PEC_XM = 1u << 2,  // node (i-1, j): affects the +x populations
    NB_PEC_XP = 1u << 3,  // node (i+1, j): affects the -x populations
    NB_PEC_YM = 1u << 4,  // node (i, j-1): affects the +y populations
    NB_PEC_YP = 1u << 5,  // node (i, j+1): affects the -y populations
};

// Relaxation of the scattered part of the zero-gradient open-edge
// extrapolation (the entering population is I_ghost + (1 - delta)(f* - I)).
constexpr double OPEN_DELTA = 1.0 / 20.0;

// Rows are padded to a multiple of this many nodes.
constexpr int ROW_ALIGN = 64;

// Lattice of one solve as the kernels see it.  Rows 0..ny-1 are the domain,
// row ny is the one-row incident-wave companion lattice.  Every population
// (or field) plane holds (ny + 1) * pitch elements.
struct Lattice {
    int nx, ny, pitch;
    size_t plane;
    const uint8_t *mask;  // [ny][pitch]
    double eps[4];        // permittivity per material id (id 3 unused)
    double eps_rest[4];   // eps - 2/3: coefficient of Ez in the rest e-population's equilibrium
};

// Contour samples (structure of arrays, n entries each).
struct ContourDev {
    int n;
    double rc;
    const int *i0, *j0;         // lower-left node of the bilinear stencil
    const double *wx, *wy;      // fractional offsets inside the cell
    const double *nxk, *nyk;    // outward unit normal
    double *acc;                // [4][n]: time sums of Ez^2, Hx^2, Hy^2, Hx*Hy
};

// Launchers (return the first HIP error).
hipError_t launch_step_f64(const Lattice &L, const double *src, double *dst, double *fields, double einc,
                           hipStream_t s);
hipError_t launch_step_neq(int precision, const Lattice &L, const void *src, void *dst, double einc, hipStream_t s);
// Fields: FP64 planes [3][plane] for precision 0, the FP32 field planes of the
// state for precisions 1 and 2.
hipError_t launch_contour(int precision, const Lattice &L, const void *fields, const ContourDev &C, hipStream_t s);
hipError_t launch_reduce(const ContourDev &C, double inv_window, double f0, double m0, double *out, hipStream_t s);
hipError_t launch_energy(int precision, const Lattice &L, const void *fields, double *partials, int nparts,
                         double *out, hipStream_t s);
int energy_partials(const Lattice &L);
hipError_t launch_fields_out(int precision, const Lattice &L, const void *fields, double *ez, double *hx, double *hy,
                             hipStream_t s);

}  // namespace jlb
