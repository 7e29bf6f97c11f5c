// Device helpers shared by the gfx950 kernel files (jlb_device.hip,
// jlb_device_f64.hip): stores, per-material coefficient picks, node
// indexing, the XCD-aware work order, the DPP wave shifts, and the FP64 node
// update (its collision is shared by the one- and two-step FP64 kernels and
// the batched engine).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include "jlb_internal.h"

namespace jlb {
namespace {

// Stores of the next state are read only in the next step.  When the state
// is larger than the 256 MB Infinity Cache they stream past the caches
// (non-temporal); when it fits, ordinary stores keep it cache-resident for
// the next step.  The choice is per launch (Lattice::stream_stores).
template <typename T> __device__ __forceinline__ void put(T *p, T v, bool stream)
{
    if (stream) __builtin_nontemporal_store(v, p);
    else *p = v;
}

constexpr int BX = 64;  // one wavefront per row segment
constexpr int BY = 4;   // four rows per block

// Material parameters by id.  Ids vary per lane; the compiler would turn a
// select among the uniform values back into an indexed vector load (whose
// wait also waits for every load issued before it, look-ahead rows
// included), so the values pass through readfirstlane first.
__device__ __forceinline__ float uniform(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ double uniform(double x)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename R> __device__ __forceinline__ R mat_pick(const double (&v)[4], int mat)
{
    const R v0 = uniform((R)v[0]), v1 = uniform((R)v[1]), v2 = uniform((R)v[2]), v3 = uniform((R)v[3]);
    return mat == 0 ? v0 : mat == 1 ? v1 : mat == 2 ? v2 : v3;
}
__device__ __forceinline__ double mat_eps(const Lattice &L, int mat) { return mat_pick<double>(L.eps, mat); }
__device__ __forceinline__ double mat_eps_rest(const Lattice &L, int mat) { return mat_pick<double>(L.eps_rest, mat); }
__device__ __forceinline__ double mat_inv_eps(const Lattice &L, int mat) { return mat_pick<double>(L.inv_eps, mat); }
// FP32 coefficients: picked among the host-rounded float copies, so the
// select runs on 32-bit values and needs no conversion per node.
__device__ __forceinline__ float mat_pick_f(const float (&v)[4], int mat)
{
    const float v0 = uniform(v[0]), v1 = uniform(v[1]), v2 = uniform(v[2]), v3 = uniform(v[3]);
    return mat == 0 ? v0 : mat == 1 ? v1 : mat == 2 ? v2 : v3;
}
__device__ __forceinline__ float mat_eps_rest_f(const Lattice &L, int mat) { return mat_pick_f(L.eps_rest_f, mat); }
__device__ __forceinline__ float mat_inv_eps_f(const Lattice &L, int mat) { return mat_pick_f(L.inv_eps_f, mat); }

// Mask index of node (i, j).
__device__ __forceinline__ size_t node(const Lattice &L, int i, int j) { return (size_t)j * L.pitch + i; }
// Index of node (i, j) in plane 0 of a row-interleaved array with row stride S.
__device__ __forceinline__ size_t at(int i, int j, size_t S) { return (size_t)j * S + i; }

// Source value of a batched solve at its step n (ramp table, then one period).
__device__ __forceinline__ double batch_incident(const SolveDesc &d, int64_t n)
{
    return n < d.ramp_end ? d.src_tab[n] : d.src_tab[d.ramp_end + n % d.T];
}

// Workgroups are handed to the eight XCDs in turn (block b on XCD b mod 8),
// and each XCD has its own L2.  Renumbering so that XCD x works through one
// contiguous range of tiles keeps the halo rows that adjacent tiles share
// inside one L2.  The map is a bijection of [0, nb).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b % NUM_XCD, k = b / NUM_XCD;
    const int per = nb / NUM_XCD, rem = nb % NUM_XCD;
    return x * per + min(x, rem) + k;
}

// Tile coordinates of this block in a 2-D grid.  A cache-resident state
// (no streaming stores) gains from XCD-contiguous tiles; a state streamed
// from HBM runs faster with every XCD on neighbouring rows (the plain order).
__device__ __forceinline__ void block_tile(const Lattice &L, int &tx, int &ty)
{
    const int nb = gridDim.x * gridDim.y;
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    const int t = L.stream_stores ? b : xcd_tile(b, nb);
    tx = t % gridDim.x;
    ty = t / gridDim.x;
}

__device__ __forceinline__ int batch_tile(const SolveDesc *D, int b, int nb, int remap)
{
    return remap ? xcd_tile(b, nb) : b;
}

// x-neighbour exchange across the wavefront with DPP wave shifts (a VALU
// move, no LDS traffic): lane k receives the value of lane k - 1
// (from_left) or of lane k + 1 (from_right); the end lanes, which have no
// such neighbour in the wavefront, receive 0 (callers load or ignore it).
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// ---------------------------------------------------------------------------
// FP64, 11 populations (arXiv 2509.22308 Sec. III, reduced TM^z form; see
// jlb_device_f64.hip).  Evaluation order and groupings match the plain
// definition so that results are reproducible to the last bits; no FMA
// contraction.
// ---------------------------------------------------------------------------

// One node's collision from the 11 populations pulled into it: the moments,
// the equilibria and f* = 2 f^eq - f into out; the node's fields (TM^z: Ez,
// Hx, Hy; TE^z in the dual storage: Hz, -Ex, -Ey) into ez, hx, hy.  Where
// the plain definition divides (by eps, 3 and 6) the update multiplies by
// the reciprocal rounded once (inv_eps per material, 1/3, 1/6): each product
// lies within one unit in the last place of the quotient, and the division
// sequence it replaces is about half of the update's instructions.
__device__ __forceinline__ void f64_collide(const Lattice &L, const double (&f)[11], double inv_eps, double eps_rest,
                                            bool conductor, double (&out)[11], double &ez, double &hx, double &hy)
{
#pragma clang fp contract(off)
    constexpr double third = 1.0 / 3.0, sixth = 1.0 / 6.0;
    const double dz = f[0] + f[1] + f[2] + (f[3] + f[4]);
    double q[11];
    if (L.te) {  // (Hz, -Ex, -Ey): the in-plane fields carry eps
        ez = dz;
        hx = (f[5] + f[6] + f[7] + (f[3] - f[4])) * inv_eps;
        hy = (f[8] + (f[9] + f[10]) + (f[2] - f[1])) * inv_eps;
        if (conductor) { hx = 0.0; hy = 0.0; }  // Ex = Ey = 0
        q[0] = ez * third;
        q[5] = eps_rest * hx;
        q[8] = eps_rest * hy;
    } else {
        ez = dz * inv_eps;
        hx = f[5] + f[6] + f[7] + (f[3] - f[4]);
        hy = f[8] + (f[9] + f[10]) + (f[2] - f[1]);
        if (conductor) ez = 0.0;  // Ez = 0
        q[0] = eps_rest * ez;
        q[5] = hx * third;
        q[8] = hy * third;
    }
    q[1] = (ez - hy) * sixth;
    q[2] = (ez + hy) * sixth;
    q[3] = (ez + hx) * sixth;
    q[4] = (ez - hx) * sixth;
    q[6] = hx * sixth;
    q[7] = hx * sixth;
    q[9] = hy * sixth;
    q[10] = hy * sixth;
#pragma unroll
    for (int k = 0; k < 11; ++k) out[k] = 2.0 * q[k] - f[k];
}

// One-step update of node (i, j) (row ny: the incident-wave companion row)
// from the state in memory.
__device__ __forceinline__ void f64_node(const Lattice &L, const double *__restrict__ src, double *__restrict__ dst,
                                         double *__restrict__ fields, double einc, int i, int j)
{
#pragma clang fp contract(off)
    const size_t P = L.plane;
    const size_t c = at(i, j, L.sf);
    const double keep = 1.0 - OPEN_DELTA;
    double f[11];
    double inv_eps = 1.0, eps_rest = 1.0 - 2.0 / 3.0;
    bool conductor = false;

    f[0] = src[0 * P + c];
    f[5] = src[5 * P + c];
    f[8] = src[8 * P + c];
    if (j == L.ny) {
        // incident-wave companion row: vacuum, uniform in y, nothing enters on the right
        f[3] = src[3 * P + c];
        f[4] = src[4 * P + c];
        f[9] = src[9 * P + c];
        f[10] = src[10 * P + c];
        if (i == 0) { f[1] = einc / 3.0; f[6] = 0.0; }
        else { f[1] = src[1 * P + c - 1]; f[6] = src[6 * P + c - 1]; }
        if (i == L.nx - 1) { f[2] = 0.0; f[7] = 0.0; }
        else { f[2] = src[2 * P + c + 1]; f[7] = src[7 * P + c + 1]; }
    } else {
        const int mat = L.mask[node(L, i, j)] & 3;
        conductor = mat == MAT_PEC;
        inv_eps = mat_inv_eps(L, mat);
        eps_rest = mat_eps_rest(L, mat);
        const size_t strip = at(i, L.ny, L.sf);
        // +x populations come from (i-1, j)
        if (i == 0) { f[1] = einc / 3.0; f[6] = 0.0; }
        else { f[1] = src[1 * P + c - 1]; f[6] = src[6 * P + c - 1]; }
        // -x populations come from (i+1, j)
        if (i == L.nx - 1) { f[2] = keep * src[2 * P + c]; f[7] = keep * src[7 * P + c]; }
        else { f[2] = src[2 * P + c + 1]; f[7] = src[7 * P + c + 1]; }
        // +y populations come from (i, j-1)
        if (j == 0) {
            f[3] = keep * src[3 * P + c] + OPEN_DELTA * src[3 * P + strip];
            f[9] = keep * src[9 * P + c] + OPEN_DELTA * src[9 * P + strip];
        } else { f[3] = src[3 * P + c - L.sf]; f[9] = src[9 * P + c - L.sf]; }
        // -y populations come from (i, j+1)
        if (j == L.ny - 1) {
            f[4] = keep * src[4 * P + c] + OPEN_DELTA * src[4 * P + strip];
            f[10] = keep * src[10 * P + c] + OPEN_DELTA * src[10 * P + strip];
        } else { f[4] = src[4 * P + c + L.sf]; f[10] = src[10 * P + c + L.sf]; }
    }
    double out[11], ez, hx, hy;
    f64_collide(L, f, inv_eps, eps_rest, conductor, out, ez, hx, hy);
#pragma unroll
    for (int k = 0; k < 11; ++k) put(&dst[k * P + c], out[k], L.stream_stores);
    if (fields) {  // row ny: the incident wave's fields (read by the far-field phasors)
        const size_t cf = at(i, j, L.sfld);
        fields[0 * P + cf] = ez;
        fields[1 * P + cf] = hx;
        fields[2 * P + cf] = hy;
    }
}

}  // namespace
}  // namespace jlb
