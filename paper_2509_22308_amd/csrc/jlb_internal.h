// Internal interface between the host driver (jlb_host.cpp) and the gfx950
// kernels (jlb_device.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jlb {

// Material id in the low two bits of a mask byte.  A conductor node (id 3)
// is updated like the others with a zero electric field (its coefficient
// 1/eps on the moment that carries the permittivity is 0).
enum : uint8_t { MAT_VACUUM = 0, MAT_REGION2 = 1, MAT_REGION3 = 2, MAT_PEC = 3 };
// The node is a corner of some contour sample's bilinear stencil.
enum : uint8_t { MASK_CONTOUR = 1u << 6 };

// Relaxation of the scattered part of the zero-gradient open-edge
// extrapolation (the entering population is I_ghost + (1 - delta)(f* - I)).
constexpr double OPEN_DELTA = 1.0 / 20.0;

// Rows are padded to a multiple of this many nodes: 64 bytes of FP32, so
// every FP32 / FP64 plane row starts 64-byte aligned, and a multiple of the
// widest vector (4 nodes) so vector accesses never leave the padded row.
constexpr int ROW_ALIGN = 16;

// Lattice of one solve as the kernels see it.  Rows 0..ny-1 are the domain,
// row ny is the one-row incident-wave companion lattice.
//
// Layout: row-interleaved planes.  Row j of the state holds, one after the
// other, the pitch-long row j of every plane, so element (q, i, j) of an
// array with row stride S sits at q * plane + j * S + i with plane = pitch.
// One lattice row is then one contiguous stretch of memory, which keeps the
// number of DRAM pages a step touches at once small.
//  * FP64 state: 11 planes of double, S = sf = 11 pitch;
//  * FP32 / BF16 state: 3 field planes of float, then 8 deviation planes of
//    float or bfloat16; float elements have row stride sf, deviation
//    elements sn (both = row bytes / element size);
//  * fields read by the contour, energy and output kernels: the FP64 field
//    array (3 planes of double, S = 3 pitch) or the state's field planes
//    (S = sf); sfld is that stride.
// The material mask is plain [ny][pitch].
struct Lattice {
    int nx, ny, pitch;
    size_t plane;         // offset between planes inside a row: pitch
    size_t sf, sn, sfld;  // row strides in elements (see above)
    const uint8_t *mask;  // [ny][pitch]
    double eps[4];        // permittivity per material id (id 3, a conductor: 1, unused)
    double eps_rest[4];   // eps - 2/3: coefficient of Ez in the rest e-population's equilibrium
    double inv_eps[4];    // 1 / eps (the FP32 / BF16 update multiplies by it)
    float inv_eps_f[4];   // FP32 / BF16: 1 / (6 eps) and 6 (eps - 2/3), rounded once on the host
    float eps_rest_f[4];  // (those states keep one sixth of the fields); conductor: 0 and 0
    int stream_stores;    // 1: write the next state past the caches (state larger than the Infinity Cache)
    int te;               // 1: TE^z, stored as (Hz, -Ex, -Ey) in the (Ez, Hx, Hy) slots
};

// Working sets above this many bytes do not stay in the 256 MB Infinity Cache
// between steps; their state stores stream past the caches.
constexpr size_t CACHE_RESIDENT_BYTES = (size_t)160 << 20;

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
                           hipStream_t s, int variant);
// Kernel variants of the FP32 / BF16 step (identical results, different
// thread-to-node mappings); chosen per device and grid by the autotuner.
enum NeqVariant {
    NEQ_DIRECT = 0,          // one node per thread, 64 x 4 blocks
    NEQ_TILE_V2 = 1,         // two / four adjacent nodes per thread, one row
    NEQ_TILE_V4 = 2,         //   per thread, 64 x 4 thread blocks
    NEQ_TILE_V2_W256 = 3,    // the same with four wavefronts side by side in x
    NEQ_TILE_V4_W256 = 4,    //   (256 x 1 and 256 x 2 thread blocks): the halo
    NEQ_TILE_V2_W256_R2 = 5, //   between wavefronts stays on one CU
    NEQ_TILE_V4_W256_R2 = 6,
    NEQ_VARIANTS = 7
};
// FP64 step variants: one node per thread in 64 x 4, 256 x 1 or 256 x 2 thread
// blocks; two adjacent nodes per thread (16-byte accesses) in 64 x 4 or
// 256 x 1 thread blocks.
enum F64Variant { F64_R4 = 0, F64_W256_R1 = 1, F64_W256_R2 = 2, F64_PAIR_R4 = 3, F64_PAIR_W256_R1 = 4, F64_VARIANTS = 5 };
// FP64 two steps per launch: state n in src -> state n + 2 in dst (src and
// dst must differ), bit for bit equal to two launch_step_f64 launches.
// fields1 / fields2 (both null, or two distinct field buffers): the field
// planes of levels n + 1 and n + 2, as launch_step_f64 writes them.
// Variants: H output rows per wavefront; HX = 4 halo columns per side (56
// output columns: 64-byte aligned strips, the least halo work; the best on
// a cache-resident state) or 8 (48 output columns: every strip's stores
// cover whole 128-byte lines; the best on a state streamed from HBM);
// registers for two or (W3) three wavefronts per SIMD; input rows loaded
// one row (two: LA2) ahead of their first use (W3: after the row before is
// done).
enum F64TwoStepVariant {
    F64_TWO_H10_X4 = 0,
    F64_TWO_H12_X4 = 1,
    F64_TWO_H12_X4_W3 = 2,
    F64_TWO_H12_X4_LA2 = 3,
    F64_TWO_H6_X8 = 4,
    F64_TWO_H8_X8 = 5,
    F64_TWO_H8_X8_LA2 = 6,
    F64_TWO_H12_X8 = 7,
    F64_TWO_STEP_VARIANTS = 8
};
hipError_t launch_step2_f64(const Lattice &L, const double *src, double *dst, double einc0, double einc1,
                            double *fields1, double *fields2, hipStream_t s, int variant);
hipError_t launch_step_neq(int precision, const Lattice &L, const void *src, void *dst, double einc, hipStream_t s,
                           int variant);
// Two steps per launch (FP32 / BF16): state n in src -> state n + 2 in dst
// (src and dst must differ); einc0 / einc1 are the source values of steps n
// and n + 1.  Variants: V adjacent nodes per lane, H rows per wavefront, HX
// halo columns at each side of a wavefront's strip (8 keeps the output
// strips 64-byte aligned).
enum TwoStepVariant {
    TWO_V1_H8_X2 = 0,
    TWO_V1_H16_X2 = 1,
    TWO_V2_H8_X2 = 2,
    TWO_V2_H16_X2 = 3,
    TWO_V1_H8_X8 = 4,
    TWO_V2_H16_X8 = 5,
    TWO_V2_H32_X8 = 6,
    TWO_V1_H8_X8_LA2 = 7,   // the same with each row's load issued two rows ahead
    TWO_V1_H4_X8_LA2 = 8,
    TWO_V1_H16_X8_LA2 = 9,
    TWO_STEP_VARIANTS = 10
};
// mid (optional): the fields at n + 1 of the contour-stencil nodes are
// written there (3 float planes, row-interleaved, row stride 3 pitch).
hipError_t launch_step2_neq(int precision, const Lattice &L, const void *src, void *dst, double einc0, double einc1,
                            float *mid, hipStream_t s, int variant);
// S steps per launch (FP32 / BF16, S = 3 or 4 by variant): state n in src ->
// state n + S in dst (src and dst must differ); einc[0..S-1] are the source
// values of steps n .. n + S - 1.  Launches need ny >= rows + S
// (hipErrorInvalidValue otherwise).
enum MultiStepVariant {
    MULTI_S4_H10_X4 = 0,  // X4: 4 halo columns per side, 56 output columns per strip
    MULTI_S4_H12_X4 = 1,
    MULTI_S4_H16_X4 = 2,
    MULTI_S3_H10_X4 = 3,
    MULTI_S3_H12_X4 = 4,
    MULTI_S4_H12_X8 = 5,  // X8: 48 output columns per strip
    MULTI_S3_H7_X4 = 6,
    MULTI_S3_H8_X4 = 7,
    MULTI_STEP_VARIANTS = 8
};
// mid (inside the window, else null): the fields at n + 1 .. n + S - 1 of the
// contour-stencil nodes, one block of 3 row-interleaved float planes (row
// stride 3 pitch) every mid_level floats.
hipError_t launch_stepm_neq(int precision, const Lattice &L, const void *src, void *dst, const double *einc,
                            float *mid, size_t mid_level, hipStream_t s, int variant);
// Contour accumulation of the levels of a multi-step launch: nmid levels from
// mid, then the state's.
hipError_t launch_contourm(const Lattice &L, const float *mid, size_t mid_level, int nmid, const void *state,
                           const ContourDev &C, hipStream_t s);
void multi_step_shape(int variant, int &depth, int &rows);
// Strip and segment counts of a multi-step variant for an nx x ny lattice.
void multi_step_grid(int variant, int nx, int ny, int &nsx, int &nsy);
// Contour accumulation of two consecutive time levels: the fields in mid
// (as written by a two-step launch), then those of the FP32 / BF16 state.
hipError_t launch_contour2(const Lattice &L, const float *mid, const void *state, const ContourDev &C, hipStream_t s);
// Fields: FP64 planes [3][plane] for precision 0, the FP32 field planes of the
// state for precisions 1 and 2.
hipError_t launch_contour(int precision, const Lattice &L, const void *fields, const ContourDev &C, hipStream_t s);
hipError_t launch_reduce(const ContourDev &C, double inv_window, double f0, double m0, double *out, hipStream_t s);
// Far field: accumulate one level's phasor terms (cw, sw = cos, sin of omega t)
// at the contour samples into dft[12][n]; then the transform into s2[nphi]
// (scale = 2 / T).
hipError_t launch_far_dft(int precision, const Lattice &L, const void *fields, const ContourDev &C, double *dft,
                          double cw, double sw, hipStream_t s);
// The stress integral with the fields of one level (not averaged): F~x, F~y, M~z.
hipError_t launch_force_now(int precision, const Lattice &L, const void *fields, const ContourDev &C, double f0,
                            double m0, double *out, hipStream_t s);
hipError_t launch_far_field(const ContourDev &C, const double *dft, double k0, double scale, int nphi, double *s2,
                            hipStream_t s);
hipError_t launch_energy(int precision, const Lattice &L, const void *fields, double *partials, int nparts,
                         double *out, hipStream_t s);
int energy_partials(const Lattice &L);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
// Device address of the library-held scratch array of the current device
// (JLB_STATIC_SCRATCH_BYTES bytes, 256-byte aligned), looked up once per device.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
hipError_t static_scratch(void **ptr);
hipError_t launch_fields_out(int precision, const Lattice &L, const void *fields, double *ez, double *hx, double *hy,
                             hipStream_t s);

// ---------------------------------------------------------------------------
// Batched engine: per-solve descriptors in device memory.  Each solve keeps
// its own step counter n on the device; the step kernels read it to pick the
// source value and the state buffers, the advance kernel increments it, so a
// captured sequence of steps can be replayed without host involvement.
// ---------------------------------------------------------------------------

struct SolveDesc {
    Lattice L;
    char *state[2];
    double *fields;          // FP64: field planes written inside the averaging window, level t at
                             // fields + (t & 1) * fields_level
    size_t fields_level;
    float *mid;              // FP32 / BF16 two-step solves: middle-level fields of the contour-stencil nodes
    const double *src_tab;   // incident values: [ramp_end] ramp steps, then [T] by n mod T
    int64_t ramp_end, T;
    int64_t n;               // steps done (device-updated)
    int64_t steps, window;
    ContourDev C;
    int precision;
    int cur;                 // buffer holding the state at step n (device-updated)
    int two;                 // 1: advanced by two-step launches
    int mdepth;              // > 0: four-step launches while four more levels remain
};

// One block of work: a tile of one resident solve.
struct Tile {
    uint32_t slot;
    uint16_t tx, ty;
};

// Tile shape of a precision / variant: columns x rows per block.
void tile_shape(int precision, int variant, int &cols, int &rows);
// remap = 1 hands XCD-contiguous tiles to the eight XCDs (cache-resident working sets).
// Single steps: the solves with two == 0.
hipError_t launch_step_batch(int precision, int variant, SolveDesc *d, const Tile *tiles, int ntiles, int remap,
                             hipStream_t s);
hipError_t launch_contour_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s);
// Two-step launches over the solves with two == 1 (precision 1 or 2): one
// wavefront per item (slot, strip tx, row segment ty) of the given variant;
// a solve with one step left takes only that step.
hipError_t launch_step2_batch(int precision, int variant, SolveDesc *d, const Tile *items, int nitems, int remap,
                              hipStream_t s);
// Strip and segment counts of a two-step variant for an nx x ny lattice.
void two_step_shape(int variant, int nx, int ny, int &nsx, int &nsy);
// FP64 two-step launches over the FP64 solves with two == 1, one wavefront
// per item (slot, strip tx, row segment ty) of the given FP64 variant; the
// strips and segments of a grid.
hipError_t launch_step2_f64_batch(int variant, SolveDesc *d, const Tile *items, int nitems, int remap, hipStream_t s);
void two_step_shape_f64(int variant, int nx, int ny, int &nsx, int &nsy);
hipError_t launch_contour2_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s);
// After a batched multi-step launch: the averaged levels of each solve in
// multi mode, in time order.
hipError_t launch_contourm_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s);
// Four-step launches (a depth-4 variant; others: hipErrorInvalidValue) over
// the two-step solves with at least mdepth levels to go ("multi mode"; the
// launch keeps the intermediate levels' contour fields in the solve's mid
// buffer when one of them is averaged); the two-step launches, their contour
// launches and advances skip those solves.
hipError_t launch_stepm_batch(int precision, int variant, SolveDesc *d, const Tile *items, int nitems, int remap,
                              hipStream_t s);
// Advances the solves with two == which by one step (which = 0) or by up
// to two (which = 1; not those in multi mode) and flips their buffers;
// which = 2 advances the solves in multi mode by mdepth.
hipError_t launch_advance(SolveDesc *d, int nslots, int which, hipStream_t s);

}  // namespace jlb
