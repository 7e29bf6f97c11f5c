// gfx950 kernels of the Janus-cylinder EM lattice Boltzmann solve.
//
// Lattice update: arXiv 2509.22308 Sec. III, Eq. (LBGK equation) with the
// equilibria of Eq. (equilibrium distribution functions), tau = 1/2.  In
// TM^z with mu_r = 1 the D3Q7 vector populations leave 11 independent
// scalars per node (the +-z populations stream in place and merge with the
// rest one; along each in-plane link one e/h combination has zero
// equilibrium and stays zero):
//   0 e_r  1 e_{+x}  2 e_{-x}  3 e_{+y}  4 e_{-y}  5 hx_r  6 hx_{+x}  7 hx_{-x}
//   8 hy_r 9 hy_{+y} 10 hy_{-y}
// with moments Dz = e_r + e_{+x} + e_{-x} + e_{+y} + e_{-y}, Ez = Dz / eps,
// Hx = hx_r + hx_{+x} + hx_{-x} + e_{+y} - e_{-y},
// Hy = hy_r + hy_{+y} + hy_{-y} + e_{-x} - e_{+x},
// and equilibria e_{+-x} = (Ez -+ Hy)/6, e_{+-y} = (Ez +- Hx)/6,
// e_r = (eps - 2/3) Ez, hx_{+-x} = Hx/6, hy_{+-y} = Hy/6, hx_r = Hx/3,
// hy_r = Hy/3.  The step is a pull: each node gathers the post-collision
// populations that stream into it, forms the moments, and stores
// f* = 2 f^eq - f.
//
// Boundaries (readings of Sec. III): populations entering through the left
// edge are the incident-wave equilibria (E_z = E_inc, H_y = -E_inc); those
// entering through the other edges extrapolate the scattered part with
// zero gradient relaxed by OPEN_DELTA against the undisturbed incident wave,
// which a one-row companion lattice (row ny) carries; a link to a perfect
// conductor reflects the opposite population with a sign change (wall at
// the link midpoint).  Conductor nodes hold nothing and are never written.
//
// Storage: FP64 keeps the 11 populations per node (176 bytes per update).
// FP32 and BF16 keep the fields (Ez, Hx, Hy) in FP32 and the deviations from
// equilibrium N_q = f_q - f_q^eq of the 8 moving populations in FP32 or
// bfloat16 (88 or 56 bytes per update): post-collision f*_q = f_q^eq - N_q,
// and the rest deviations follow from the moments, which every equilibrium
// reproduces: N_er = -(N_{e+x} + N_{e-x} + N_{e+y} + N_{e-y}) and likewise
// for hx and hy.  The large rest population (eps - 2/3) Ez therefore never
// passes through a narrow format.
//
// No MFMA: the step is a stencil with about 0.3 flop per byte.
#include <hip/hip_runtime.h>

#include "jlb_internal.h"

namespace jlb {

namespace {

constexpr int BX = 64;  // one wavefront per row segment
constexpr int BY = 4;   // four rows per block

__device__ __forceinline__ size_t node(const Lattice &L, int i, int j) { return (size_t)j * L.pitch + i; }

// ---------------------------------------------------------------------------
// FP64, 11 populations.  Evaluation order and groupings match the plain
// definition so that results are reproducible to the last bits; no FMA
// contraction.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BX *BY) void k_step_f64(Lattice L, const double *__restrict__ src,
                                                      double *__restrict__ dst, double *__restrict__ fields,
                                                      double einc)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    if (i >= L.nx || j > L.ny) return;
    const size_t P = L.plane;
    const size_t c = node(L, i, j);
    const double keep = 1.0 - OPEN_DELTA;
    double f[11];
    double eps = 1.0, eps_rest = 1.0 - 2.0 / 3.0;

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
        const uint8_t m = L.mask[c];
        const int mat = m & 3;
        if (mat == MAT_PEC) return;
        eps = L.eps[mat];
        eps_rest = L.eps_rest[mat];
        const size_t strip = node(L, i, L.ny);
        // +x populations come from (i-1, j)
        if (i == 0) { f[1] = einc / 3.0; f[6] = 0.0; }
        else if (m & NB_PEC_XM) { f[1] = -src[2 * P + c]; f[6] = -src[7 * P + c]; }
        else { f[1] = src[1 * P + c - 1]; f[6] = src[6 * P + c - 1]; }
        // -x populations come from (i+1, j)
        if (i == L.nx - 1) { f[2] = keep * src[2 * P + c]; f[7] = keep * src[7 * P + c]; }
        else if (m & NB_PEC_XP) { f[2] = -src[1 * P + c]; f[7] = -src[6 * P + c]; }
        else { f[2] = src[2 * P + c + 1]; f[7] = src[7 * P + c + 1]; }
        // +y populations come from (i, j-1)
        if (j == 0) {
            f[3] = keep * src[3 * P + c] + OPEN_DELTA * src[3 * P + strip];
            f[9] = keep * src[9 * P + c] + OPEN_DELTA * src[9 * P + strip];
        } else if (m & NB_PEC_YM) { f[3] = -src[4 * P + c]; f[9] = -src[10 * P + c]; }
        else { f[3] = src[3 * P + c - L.pitch]; f[9] = src[9 * P + c - L.pitch]; }
        // -y populations come from (i, j+1)
        if (j == L.ny - 1) {
            f[4] = keep * src[4 * P + c] + OPEN_DELTA * src[4 * P + strip];
            f[10] = keep * src[10 * P + c] + OPEN_DELTA * src[10 * P + strip];
        } else if (m & NB_PEC_YP) { f[4] = -src[3 * P + c]; f[10] = -src[9 * P + c]; }
        else { f[4] = src[4 * P + c + L.pitch]; f[10] = src[10 * P + c + L.pitch]; }
    }

    const double dz = f[0] + f[1] + f[2] + (f[3] + f[4]);
    const double ez = dz / eps;
    const double hx = f[5] + f[6] + f[7] + (f[3] - f[4]);
    const double hy = f[8] + (f[9] + f[10]) + (f[2] - f[1]);
    double q[11];
    q[0] = eps_rest * ez;
    q[1] = (ez - hy) / 6.0;
    q[2] = (ez + hy) / 6.0;
    q[3] = (ez + hx) / 6.0;
    q[4] = (ez - hx) / 6.0;
    q[5] = hx / 3.0;
    q[6] = hx / 6.0;
    q[7] = hx / 6.0;
    q[8] = hy / 3.0;
    q[9] = hy / 6.0;
    q[10] = hy / 6.0;
#pragma unroll
    for (int k = 0; k < 11; ++k) dst[k * P + c] = 2.0 * q[k] - f[k];
    if (fields && j < L.ny) {
        fields[0 * P + c] = ez;
        fields[1 * P + c] = hx;
        fields[2 * P + c] = hy;
    }
}

// ---------------------------------------------------------------------------
// FP32 / BF16: fields + deviations from equilibrium.
// State planes: F = {Ez, Hx, Hy} (float), N = 8 moving deviations in the
// order {e+x, e-x, e+y, e-y, hx+x, hx-x, hy+y, hy-y}.
// ---------------------------------------------------------------------------

enum { N_EPX = 0, N_EMX, N_EPY, N_EMY, N_HXPX, N_HXMX, N_HYPY, N_HYMY };

template <typename T> __device__ __forceinline__ float ld(const T *p) { return (float)*p; }
template <typename T> __device__ __forceinline__ void st(T *p, float v) { *p = (T)v; }

template <typename NeqT>
struct NeqState {
    float *F;     // [3][plane]
    NeqT *N;      // [8][plane]
};

template <typename NeqT>
__device__ __forceinline__ NeqState<NeqT> neq_view(void *base, size_t plane)
{
    NeqState<NeqT> s;
    s.F = reinterpret_cast<float *>(base);
    s.N = reinterpret_cast<NeqT *>(s.F + 3 * plane);
    return s;
}

template <typename NeqT>
__global__ __launch_bounds__(BX *BY) void k_step_neq(Lattice L, const void *__restrict__ srcv,
                                                      void *__restrict__ dstv, float einc)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    if (i >= L.nx || j > L.ny) return;
    const size_t P = L.plane;
    const NeqState<NeqT> S = neq_view<NeqT>(const_cast<void *>(srcv), P);
    const NeqState<NeqT> D = neq_view<NeqT>(dstv, P);
    const size_t c = node(L, i, j);
    const float keep = (float)(1.0 - OPEN_DELTA);
    const float delta = (float)OPEN_DELTA;
    const float sixth = 1.0f / 6.0f, third = 1.0f / 3.0f;

    uint8_t m = 0;
    float eps = 1.0f, eps_rest = (float)(1.0 - 2.0 / 3.0);
    const bool strip_row = (j == L.ny);
    if (!strip_row) {
        m = L.mask[c];
        const int mat = m & 3;
        if (mat == MAT_PEC) return;
        eps = (float)L.eps[mat];
        eps_rest = (float)L.eps_rest[mat];
    }

    // own fields and deviations at time n
    const float ez0 = S.F[0 * P + c], hx0 = S.F[1 * P + c], hy0 = S.F[2 * P + c];
    float n0[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) n0[k] = ld(&S.N[k * P + c]);
    // own post-collision moving populations (used by edges and conductor links)
    const float s_epx = (ez0 - hy0) * sixth - n0[N_EPX];
    const float s_emx = (ez0 + hy0) * sixth - n0[N_EMX];
    const float s_epy = (ez0 + hx0) * sixth - n0[N_EPY];
    const float s_emy = (ez0 - hx0) * sixth - n0[N_EMY];
    const float s_hxpx = hx0 * sixth - n0[N_HXPX];
    const float s_hxmx = hx0 * sixth - n0[N_HXMX];
    const float s_hypy = hy0 * sixth - n0[N_HYPY];
    const float s_hymy = hy0 * sixth - n0[N_HYMY];
    // rest populations stream in place: f*_r = f_r^eq - N_r with the sum rules
    const float r_e = eps_rest * ez0 + (n0[N_EPX] + n0[N_EMX] + n0[N_EPY] + n0[N_EMY]);
    const float r_hx = hx0 * third + (n0[N_HXPX] + n0[N_HXMX] + n0[N_EPY] - n0[N_EMY]);
    const float r_hy = hy0 * third + (n0[N_HYPY] + n0[N_HYMY] - n0[N_EPX] + n0[N_EMX]);

    float e_px, hx_px, e_mx, hx_mx, e_py, hy_py, e_my, hy_my;
    // +x from (i-1, j)
    if (i == 0) { e_px = einc * third; hx_px = 0.0f; }
    else if (m & NB_PEC_XM) { e_px = -s_emx; hx_px = -s_hxmx; }
    else {
        const size_t s = c - 1;
        const float ez = S.F[0 * P + s], hx = S.F[1 * P + s], hy = S.F[2 * P + s];
        e_px = (ez - hy) * sixth - ld(&S.N[N_EPX * P + s]);
        hx_px = hx * sixth - ld(&S.N[N_HXPX * P + s]);
    }
    // -x from (i+1, j)
    if (i == L.nx - 1) {
        if (strip_row) { e_mx = 0.0f; hx_mx = 0.0f; }
        else { e_mx = keep * s_emx; hx_mx = keep * s_hxmx; }
    } else if (m & NB_PEC_XP) { e_mx = -s_epx; hx_mx = -s_hxpx; }
    else {
        const size_t s = c + 1;
        const float ez = S.F[0 * P + s], hx = S.F[1 * P + s], hy = S.F[2 * P + s];
        e_mx = (ez + hy) * sixth - ld(&S.N[N_EMX * P + s]);
        hx_mx = hx * sixth - ld(&S.N[N_HXMX * P + s]);
    }
    if (strip_row) {
        // uniform in y: the +-y populations stay in their node
        e_py = s_epy; hy_py = s_hypy; e_my = s_emy; hy_my = s_hymy;
    } else {
        const size_t strip = node(L, i, L.ny);
        float i_epy = 0.0f, i_hypy = 0.0f, i_emy = 0.0f, i_hymy = 0.0f;
        if (j == 0 || j == L.ny - 1) {
            const float ez = S.F[0 * P + strip], hx = S.F[1 * P + strip], hy = S.F[2 * P + strip];
            i_epy = (ez + hx) * sixth - ld(&S.N[N_EPY * P + strip]);
            i_hypy = hy * sixth - ld(&S.N[N_HYPY * P + strip]);
            i_emy = (ez - hx) * sixth - ld(&S.N[N_EMY * P + strip]);
            i_hymy = hy * sixth - ld(&S.N[N_HYMY * P + strip]);
        }
        // +y from (i, j-1)
        if (j == 0) { e_py = keep * s_epy + delta * i_epy; hy_py = keep * s_hypy + delta * i_hypy; }
        else if (m & NB_PEC_YM) { e_py = -s_emy; hy_py = -s_hymy; }
        else {
            const size_t s = c - L.pitch;
            const float ez = S.F[0 * P + s], hx = S.F[1 * P + s];
            e_py = (ez + hx) * sixth - ld(&S.N[N_EPY * P + s]);
            hy_py = S.F[2 * P + s] * sixth - ld(&S.N[N_HYPY * P + s]);
        }
        // -y from (i, j+1)
        if (j == L.ny - 1) { e_my = keep * s_emy + delta * i_emy; hy_my = keep * s_hymy + delta * i_hymy; }
        else if (m & NB_PEC_YP) { e_my = -s_epy; hy_my = -s_hypy; }
        else {
            const size_t s = c + L.pitch;
            const float ez = S.F[0 * P + s], hx = S.F[1 * P + s];
            e_my = (ez - hx) * sixth - ld(&S.N[N_EMY * P + s]);
            hy_my = S.F[2 * P + s] * sixth - ld(&S.N[N_HYMY * P + s]);
        }
    }

    const float dz = r_e + e_px + e_mx + (e_py + e_my);
    const float ez = dz / eps;
    const float hx = r_hx + hx_px + hx_mx + (e_py - e_my);
    const float hy = r_hy + (hy_py + hy_my) + (e_mx - e_px);
    D.F[0 * P + c] = ez;
    D.F[1 * P + c] = hx;
    D.F[2 * P + c] = hy;
    st(&D.N[N_EPX * P + c], e_px - (ez - hy) * sixth);
    st(&D.N[N_EMX * P + c], e_mx - (ez + hy) * sixth);
    st(&D.N[N_EPY * P + c], e_py - (ez + hx) * sixth);
    st(&D.N[N_EMY * P + c], e_my - (ez - hx) * sixth);
    st(&D.N[N_HXPX * P + c], hx_px - hx * sixth);
    st(&D.N[N_HXMX * P + c], hx_mx - hx * sixth);
    st(&D.N[N_HYPY * P + c], hy_py - hy * sixth);
    st(&D.N[N_HYMY * P + c], hy_my - hy * sixth);
}

// ---------------------------------------------------------------------------
// Contour sampling (Sec. II.B): bilinear fields at each sample, time sums of
// Ez^2, Hx^2, Hy^2 and Hx Hy in FP64.  One thread per sample, no atomics.
// ---------------------------------------------------------------------------

__global__ void k_contour_f64(Lattice L, const double *__restrict__ fld, ContourDev C)
{
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.n) return;
    const size_t P = L.plane;
    const size_t c00 = node(L, C.i0[k], C.j0[k]);
    const size_t c10 = c00 + L.pitch;
    const double fx = C.wx[k], fy = C.wy[k];
    const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy), w10 = (1.0 - fx) * fy, w11 = fx * fy;
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double *p = fld + a * P;
        v[a] = w00 * p[c00] + w01 * p[c00 + 1] + w10 * p[c10] + w11 * p[c10 + 1];
    }
    C.acc[0 * C.n + k] += v[0] * v[0];
    C.acc[1 * C.n + k] += v[1] * v[1];
    C.acc[2 * C.n + k] += v[2] * v[2];
    C.acc[3 * C.n + k] += v[1] * v[2];
}

__global__ void k_contour_f32(Lattice L, const float *__restrict__ fld, ContourDev C)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.n) return;
    const size_t P = L.plane;
    const size_t c00 = node(L, C.i0[k], C.j0[k]);
    const size_t c10 = c00 + L.pitch;
    const float fx = (float)C.wx[k], fy = (float)C.wy[k];
    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy), w10 = (1.0f - fx) * fy, w11 = fx * fy;
    float v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *p = fld + a * P;
        v[a] = w00 * p[c00] + w01 * p[c00 + 1] + w10 * p[c10] + w11 * p[c10 + 1];
    }
    C.acc[0 * C.n + k] += (double)(v[0] * v[0]);
    C.acc[1 * C.n + k] += (double)(v[1] * v[1]);
    C.acc[2 * C.n + k] += (double)(v[2] * v[2]);
    C.acc[3 * C.n + k] += (double)(v[1] * v[2]);
}

// ---------------------------------------------------------------------------
// Contour reduction (Sec. II.B, Eqs. force and torque): time-averaged stress
// T_xx = (Hx^2 - Hy^2 - Ez^2)/2, T_yy = (Hy^2 - Hx^2 - Ez^2)/2, T_xy = Hx Hy;
// F = sum_k w T.n_k, M_z = sum_k w R_c (n_x (T.n)_y - n_y (T.n)_x), w = 2 pi R_c / N.
// One block; per-thread strided sums, then a wavefront butterfly and a fixed
// order across the block's wavefronts, all in FP64.
// ---------------------------------------------------------------------------

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce(ContourDev C, double inv_window, double f0, double m0,
                                                        double *out)
{
    __shared__ double part[3][RED_THREADS / 64];
    const int t = threadIdx.x;
    const double w = 2.0 * M_PI * C.rc / C.n;
    double fx = 0.0, fy = 0.0, tz = 0.0;
    for (int k = t; k < C.n; k += RED_THREADS) {
        const double e2 = C.acc[0 * C.n + k] * inv_window, x2 = C.acc[1 * C.n + k] * inv_window;
        const double y2 = C.acc[2 * C.n + k] * inv_window, xy = C.acc[3 * C.n + k] * inv_window;
        const double txx = 0.5 * (x2 - y2 - e2);
        const double tyy = 0.5 * (y2 - x2 - e2);
        const double nx = C.nxk[k], ny = C.nyk[k];
        const double tx = txx * nx + xy * ny;
        const double ty = xy * nx + tyy * ny;
        fx += w * tx;
        fy += w * ty;
        tz += w * C.rc * (nx * ty - ny * tx);
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    tz = wave_sum(tz);
    if ((t & 63) == 0) {
        part[0][t >> 6] = fx;
        part[1][t >> 6] = fy;
        part[2][t >> 6] = tz;
    }
    __syncthreads();
    if (t == 0) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < RED_THREADS / 64; ++b) s[a] += part[a][b];
        out[0] = s[0] / f0;
        out[1] = s[1] / f0;
        out[2] = s[2] / m0;
        out[3] = s[0];
        out[4] = s[1];
        out[5] = s[2];
    }
}

// ---------------------------------------------------------------------------
// Field energy sum (eps Ez^2 + Hx^2 + Hy^2) / 2 over the domain rows: one
// partial per block, then one fixed-order pass.
// ---------------------------------------------------------------------------

constexpr int EN_THREADS = 256;
constexpr int EN_ROWS = 4;

template <typename FT>
__global__ __launch_bounds__(EN_THREADS) void k_energy_partial(Lattice L, const FT *__restrict__ fld,
                                                               double *partials)
{
    __shared__ double part[EN_THREADS / 64];
    const int t = threadIdx.x;
    const size_t P = L.plane;
    double s = 0.0;
    for (int r = 0; r < EN_ROWS; ++r) {
        const int j = blockIdx.y * EN_ROWS + r;
        if (j >= L.ny) break;
        for (int i = blockIdx.x * EN_THREADS + t; i < L.nx && i < (int)(blockIdx.x + 1) * EN_THREADS; i += EN_THREADS) {
            const size_t c = node(L, i, j);
            const int mat = L.mask[c] & 3;
            if (mat == MAT_PEC) continue;
            const double ez = fld[c], hx = fld[P + c], hy = fld[2 * P + c];
            s += 0.5 * (L.eps[mat] * ez * ez + hx * hx + hy * hy);
        }
    }
    s = wave_sum(s);
    if ((t & 63) == 0) part[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        double v = 0.0;
        for (int b = 0; b < EN_THREADS / 64; ++b) v += part[b];
        partials[blockIdx.y * gridDim.x + blockIdx.x] = v;
    }
}

__global__ void k_energy_final(const double *partials, int n, double *out)
{
    __shared__ double part[RED_THREADS / 64];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int k = t; k < n; k += RED_THREADS) s += partials[k];
    s = wave_sum(s);
    if ((t & 63) == 0) part[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        double v = 0.0;
        for (int b = 0; b < RED_THREADS / 64; ++b) v += part[b];
        *out = v;
    }
}

template <typename FT>
__global__ void k_fields_out(Lattice L, const FT *__restrict__ fld, double *ez, double *hx, double *hy)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= L.nx || j >= L.ny) return;
    const size_t P = L.plane;
    const size_t c = node(L, i, j);
    const size_t o = (size_t)j * L.nx + i;
    ez[o] = (double)fld[c];
    hx[o] = (double)fld[P + c];
    hy[o] = (double)fld[2 * P + c];
}

dim3 step_grid(const Lattice &L) { return dim3((L.nx + BX - 1) / BX, (L.ny + 1 + BY - 1) / BY); }

}  // namespace

hipError_t launch_step_f64(const Lattice &L, const double *src, double *dst, double *fields, double einc,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_step_f64, step_grid(L), dim3(BX, BY), 0, s, L, src, dst, fields, einc);
    return hipGetLastError();
}

hipError_t launch_step_neq(int precision, const Lattice &L, const void *src, void *dst, double einc, hipStream_t s)
{
    if (precision == 1)
        hipLaunchKernelGGL(k_step_neq<float>, step_grid(L), dim3(BX, BY), 0, s, L, src, dst, (float)einc);
    else
        hipLaunchKernelGGL(k_step_neq<__bf16>, step_grid(L), dim3(BX, BY), 0, s, L, src, dst, (float)einc);
    return hipGetLastError();
}

hipError_t launch_contour(int precision, const Lattice &L, const void *fields, const ContourDev &C, hipStream_t s)
{
    const int threads = 128;
    const int blocks = (C.n + threads - 1) / threads;
    if (precision == 0)
        hipLaunchKernelGGL(k_contour_f64, dim3(blocks), dim3(threads), 0, s, L, (const double *)fields, C);
    else
        hipLaunchKernelGGL(k_contour_f32, dim3(blocks), dim3(threads), 0, s, L, (const float *)fields, C);
    return hipGetLastError();
}

hipError_t launch_reduce(const ContourDev &C, double inv_window, double f0, double m0, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, s, C, inv_window, f0, m0, out);
    return hipGetLastError();
}

int energy_partials(const Lattice &L)
{
    return ((L.nx + EN_THREADS - 1) / EN_THREADS) * ((L.ny + EN_ROWS - 1) / EN_ROWS);
}

hipError_t launch_energy(int precision, const Lattice &L, const void *fields, double *partials, int nparts,
                         double *out, hipStream_t s)
{
    dim3 grid((L.nx + EN_THREADS - 1) / EN_THREADS, (L.ny + EN_ROWS - 1) / EN_ROWS);
    if (precision == 0)
        hipLaunchKernelGGL(k_energy_partial<double>, grid, dim3(EN_THREADS), 0, s, L, (const double *)fields, partials);
    else
        hipLaunchKernelGGL(k_energy_partial<float>, grid, dim3(EN_THREADS), 0, s, L, (const float *)fields, partials);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(RED_THREADS), 0, s, partials, nparts, out);
    return hipGetLastError();
}

hipError_t launch_fields_out(int precision, const Lattice &L, const void *fields, double *ez, double *hx, double *hy,
                             hipStream_t s)
{
    dim3 grid((L.nx + 255) / 256, L.ny);
    if (precision == 0)
        hipLaunchKernelGGL(k_fields_out<double>, grid, dim3(256), 0, s, L, (const double *)fields, ez, hx, hy);
    else
        hipLaunchKernelGGL(k_fields_out<float>, grid, dim3(256), 0, s, L, (const float *)fields, ez, hx, hy);
    return hipGetLastError();
}

}  // namespace jlb
