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
// which a one-row companion lattice (row ny) carries.  A perfect conductor
// (Sec. II: E_z^tot = 0) is the update's limit of infinite permittivity: its
// nodes are updated like every other node with the electric field set to
// zero (the coefficient 1/eps of the moment that carries the permittivity is
// 0), so the wall sits on the conductor nodes.
//
// Storage: FP64 keeps the 11 populations per node (176 bytes per update).
// FP32 and BF16 keep one sixth of the fields, (Ez, Hx, Hy) / 6, in FP32 and
// the deviations from equilibrium N_q = f_q - f_q^eq of the 8 moving
// populations in FP32 or bfloat16 (88 or 56 bytes per update): a moving
// equilibrium is then a plain sum of stored fields (e.g. f^eq_{e+x} =
// (Ez - Hy) / 6), so post-collision f*_q = f_q^eq - N_q needs no multiply, and
// the factors 1/6 and 6 go into the per-material moment and rest-equilibrium
// coefficients.  The rest deviations follow from the moments, which every
// equilibrium reproduces: N_er = -(N_{e+x} + N_{e-x} + N_{e+y} + N_{e-y}) and
// likewise for hx and hy.  The large rest population (eps - 2/3) Ez
// therefore never passes through a narrow format.  Readers of the FP32
// field planes (contour sums, far field, energy, field output) scale by 6.
//
// TE^z (Hz, Ex, Ey; the polarisation the paper leaves for later, Sec. I) is
// the same update under the vacuum duality E -> H, H -> -E: the state holds
// (Hz, -Ex, -Ey) in the (Ez, Hx, Hy) slots and the populations accordingly,
// and the permittivity moves to the in-plane fields (moments eps Ex, eps Ey;
// rest equilibria Hz/3 and (eps - 2/3) Ex, (eps - 2/3) Ey), so a conductor
// node holds Ex = Ey = 0.  Source, open edges, companion row, stress sums and
// far-field phasors are unchanged in the dual storage.
//
// No MFMA: the step is a stencil with about 0.3 flop per byte.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "jlb_device_common.h"
#include "jlb_internal.h"

namespace jlb {

namespace {


// ---------------------------------------------------------------------------
// FP32 / BF16: fields + deviations from equilibrium.
// State planes: F = {Ez, Hx, Hy} (float), N = 8 moving deviations in the
// order {e+x, e-x, e+y, e-y, hx+x, hx-x, hy+y, hy-y}.
// ---------------------------------------------------------------------------

enum { N_EPX = 0, N_EMX, N_EPY, N_EMY, N_HXPX, N_HXMX, N_HYPY, N_HYMY };

template <typename T> __device__ __forceinline__ float ld(const T *p) { return (float)*p; }
template <typename T> __device__ __forceinline__ void st(T *p, float v, bool stream) { put(p, (T)v, stream); }

constexpr float SIXTH = 1.0f / 6.0f;
// Physical fields per stored field: FP32 / BF16 states keep one sixth of them.
template <typename FT> __device__ __forceinline__ double field_scale() { return sizeof(FT) == 4 ? 6.0 : 1.0; }
constexpr float THIRD = 1.0f / 3.0f;

// Fields and deviations of one node at time n.
struct NodeData {
    float ez, hx, hy;
    float n[8];
};

// What a neighbour contributes to a pull: its fields and the two deviations
// of the populations that stream from it towards the node.
struct Side {
    float ez, hx, hy, na, nb;
};

template <typename NeqT>
__device__ __forceinline__ NodeData load_node(const float *F, const NeqT *N, size_t P, size_t cf, size_t cn)
{
    NodeData d;
    d.ez = F[cf];
    d.hx = F[P + cf];
    d.hy = F[2 * P + cf];
#pragma unroll
    for (int k = 0; k < 8; ++k) d.n[k] = ld(&N[k * P + cn]);
    return d;
}

template <typename NeqT>
__device__ __forceinline__ Side load_side(const float *F, const NeqT *N, size_t P, size_t cf, size_t cn, int qa,
                                          int qb)
{
    Side s;
    s.ez = F[cf];
    s.hx = F[P + cf];
    s.hy = F[2 * P + cf];
    s.na = ld(&N[qa * P + cn]);
    s.nb = ld(&N[qb * P + cn]);
    return s;
}

// Material coefficients of one node's update.  TM^z: the z field carries the
// permittivity (Dz = eps Ez, rest equilibrium (eps - 2/3) Ez, in-plane rests
// H/3).  TE^z in the dual storage: the in-plane fields carry it and the z
// field's rest is Hz/3.  With the stored fields one sixth of the physical
// ones, a carries a factor 1/6 and c a factor 6: inv_eps6 = 1 / (6 eps),
// eps_rest6 = 6 (eps - 2/3); a conductor node has inv_eps6 = 0 (its
// electric field is zero) and eps_rest6 = 0.
struct Coef {
    float az, axy;  // stored field = moment sum * a
    float cz, cxy;  // rest equilibrium = c * stored field
};
__device__ __forceinline__ Coef coef_tm(float inv_eps6, float eps_rest6)
{
    return Coef{inv_eps6, SIXTH, eps_rest6, 2.0f};
}
__device__ __forceinline__ Coef coef_te(float inv_eps6, float eps_rest6)
{
    return Coef{SIXTH, inv_eps6, 2.0f, eps_rest6};
}
__device__ __forceinline__ Coef coef_of(const Lattice &L, float inv_eps6, float eps_rest6)
{
    return L.te ? coef_te(inv_eps6, eps_rest6) : coef_tm(inv_eps6, eps_rest6);
}
// TEM: the polarisation fixed when the kernel is compiled (0 TM^z, 1 TE^z),
// which spares the per-node choice, or read from the lattice (2).
template <int TEM>
__device__ __forceinline__ Coef coef_pick(const Lattice &L, float inv_eps6, float eps_rest6)
{
    if constexpr (TEM == 0) return coef_tm(inv_eps6, eps_rest6);
    else if constexpr (TEM == 1) return coef_te(inv_eps6, eps_rest6);
    else return coef_of(L, inv_eps6, eps_rest6);
}

// The post-collision pair a node sends along an axis: the e population and
// the h population of that direction, f* = f^eq - N.  "up" is what the row
// above pulls (+y), "down" what the row below pulls (-y), "east" what the
// node to the right pulls (+x), "west" what the node to the left pulls (-x).
struct Pair {
    float e, h;
};
// (stored fields are one sixth of the physical ones: f^eq is a plain sum)
__device__ __forceinline__ float up_e(const Side &s) { return (s.ez + s.hx) - s.na; }
__device__ __forceinline__ float up_h(const Side &s) { return s.hy - s.nb; }
__device__ __forceinline__ float down_e(const Side &s) { return (s.ez - s.hx) - s.na; }
__device__ __forceinline__ float down_h(const Side &s) { return s.hy - s.nb; }
__device__ __forceinline__ float up_e(const Pair &p) { return p.e; }
__device__ __forceinline__ float up_h(const Pair &p) { return p.h; }
__device__ __forceinline__ float down_e(const Pair &p) { return p.e; }
__device__ __forceinline__ float down_h(const Pair &p) { return p.h; }

// One node's update from its own data and the populations pulled across its
// four links (interior values; edges and the companion row replace some of
// them here).  `inc_lo` / `inc_hi` stand for the incident-wave
// companion node of the same column, as a Side (fields + N_{e+y}, N_{hy+y} /
// N_{e-y}, N_{hy-y}) or as its up / down Pair, for the bottom / top rows.
template <bool STRIP, typename Inc>
__device__ __forceinline__ void neq_pulled(const Lattice &L, int i, int j, uint8_t m, const Coef &k,
                                           const NodeData &o, float e_px, float hx_px, float e_mx, float hx_mx,
                                           float e_py, float hy_py, float e_my, float hy_my, const Inc &inc_lo,
                                           const Inc &inc_hi, float einc, NodeData &out)
{
    // no FMA contraction: every kernel variant that inlines this core must
    // round the same operations the same way
#pragma clang fp contract(off)
    const float keep = (float)(1.0 - OPEN_DELTA);
    const float delta = (float)OPEN_DELTA;
    // rest populations stream in place: f*_r = f_r^eq - N_r with the sum rules
    const float r_e = k.cz * o.ez + (o.n[N_EPX] + o.n[N_EMX] + o.n[N_EPY] + o.n[N_EMY]);
    const float r_hx = o.hx * k.cxy + (o.n[N_HXPX] + o.n[N_HXMX] + o.n[N_EPY] - o.n[N_EMY]);
    const float r_hy = o.hy * k.cxy + (o.n[N_HYPY] + o.n[N_HYMY] - o.n[N_EPX] + o.n[N_EMX]);

    // edges and the companion row replace some pulls (most wavefronts have
    // no such node and skip this block)
    if (STRIP || i == 0 || i == L.nx - 1 || j == 0 || j == L.ny - 1) {
        // own post-collision moving populations
        const float s_epx = (o.ez - o.hy) - o.n[N_EPX];
        const float s_emx = (o.ez + o.hy) - o.n[N_EMX];
        const float s_epy = (o.ez + o.hx) - o.n[N_EPY];
        const float s_emy = (o.ez - o.hx) - o.n[N_EMY];
        const float s_hxpx = o.hx - o.n[N_HXPX];
        const float s_hxmx = o.hx - o.n[N_HXMX];
        const float s_hypy = o.hy - o.n[N_HYPY];
        const float s_hymy = o.hy - o.n[N_HYMY];
        if (i == 0) { e_px = einc * THIRD; hx_px = 0.0f; }
        if (i == L.nx - 1) {
            if (STRIP) { e_mx = 0.0f; hx_mx = 0.0f; }
            else { e_mx = keep * s_emx; hx_mx = keep * s_hxmx; }
        }
        if (STRIP) {
            // uniform in y: the +-y populations stay in their node
            e_py = s_epy; hy_py = s_hypy; e_my = s_emy; hy_my = s_hymy;
        } else {
            if (j == 0) {
                e_py = keep * s_epy + delta * up_e(inc_lo);
                hy_py = keep * s_hypy + delta * up_h(inc_lo);
            }
            if (j == L.ny - 1) {
                e_my = keep * s_emy + delta * down_e(inc_hi);
                hy_my = keep * s_hymy + delta * down_h(inc_hi);
            }
        }
    }

    const float dz = r_e + e_px + e_mx + (e_py + e_my);
    const float ez = dz * k.az;
    const float hx = (r_hx + hx_px + hx_mx + (e_py - e_my)) * k.axy;
    const float hy = (r_hy + (hy_py + hy_my) + (e_mx - e_px)) * k.axy;
    out.ez = ez;
    out.hx = hx;
    out.hy = hy;
    out.n[N_EPX] = e_px - (ez - hy);
    out.n[N_EMX] = e_mx - (ez + hy);
    out.n[N_EPY] = e_py - (ez + hx);
    out.n[N_EMY] = e_my - (ez - hx);
    out.n[N_HXPX] = hx_px - hx;
    out.n[N_HXMX] = hx_mx - hx;
    out.n[N_HYPY] = hy_py - hy;
    out.n[N_HYMY] = hy_my - hy;
}

// One node's update from its own data and the four sides (fields and the two
// deviations of the populations it pulls): the interior pulls, then the core.
template <bool STRIP>
__device__ __forceinline__ void neq_core(const Lattice &L, int i, int j, uint8_t m, const Coef &k,
                                         const NodeData &o, const Side &l, const Side &r, const Side &b, const Side &t,
                                         const Side &inc_lo, const Side &inc_hi, float einc, NodeData &out)
{
#pragma clang fp contract(off)
    // pulls across interior links: the neighbour's post-collision population
    const float e_px = (l.ez - l.hy) - l.na, hx_px = l.hx - l.nb;  // +x from (i-1, j)
    const float e_mx = (r.ez + r.hy) - r.na, hx_mx = r.hx - r.nb;  // -x from (i+1, j)
    const float e_py = up_e(b), hy_py = up_h(b);                                    // +y from (i, j-1)
    const float e_my = down_e(t), hy_my = down_h(t);                                // -y from (i, j+1)
    neq_pulled<STRIP>(L, i, j, m, k, o, e_px, hx_px, e_mx, hx_mx, e_py, hy_py, e_my, hy_my, inc_lo, inc_hi, einc, out);
}

template <typename NeqT>
__device__ __forceinline__ void store_node(float *F, NeqT *N, size_t P, size_t cf, size_t cn, const NodeData &d,
                                           bool stream)
{
    put(&F[cf], d.ez, stream);
    put(&F[P + cf], d.hx, stream);
    put(&F[2 * P + cf], d.hy, stream);
#pragma unroll
    for (int k = 0; k < 8; ++k) st(&N[k * P + cn], d.n[k], stream);
}

// Sides along x of node (i, j) and the material parameters.
template <typename NeqT>
__device__ __forceinline__ void node_setup(const Lattice &L, const float *F, const NeqT *N, int i, int j, size_t cf,
                                           size_t cn, uint8_t &m, float &inv_eps, float &eps_rest, Side &l, Side &r)
{
    const size_t P = L.plane;
    m = 0;
    inv_eps = SIXTH;  // vacuum, scaled as the stored coefficients
    eps_rest = 2.0f;
    if (j < L.ny) {
        m = L.mask[node(L, i, j)];
        const int mat = m & 3;
        inv_eps = mat_inv_eps_f(L, mat);
        eps_rest = mat_eps_rest_f(L, mat);
    }
    if (i > 0) l = load_side(F, N, P, cf - 1, cn - 1, N_EPX, N_HXPX);
    if (i < L.nx - 1) r = load_side(F, N, P, cf + 1, cn + 1, N_EMX, N_HXMX);
}

template <typename NeqT>
__device__ __forceinline__ void load_incident_sides(const Lattice &L, const float *F, const NeqT *N, int i, int j,
                                                    Side &inc_lo, Side &inc_hi)
{
    const size_t P = L.plane;
    const size_t sf = at(i, L.ny, L.sf), sn = at(i, L.ny, L.sn);
    if (j == 0) inc_lo = load_side(F, N, P, sf, sn, N_EPY, N_HYPY);
    if (j == L.ny - 1) inc_hi = load_side(F, N, P, sf, sn, N_EMY, N_HYMY);
}

// ---------------------------------------------------------------------------
// FP32 / BF16 kernels.  State planes: F = {Ez, Hx, Hy} (float), N = 8 moving
// deviations in the order {e+x, e-x, e+y, e-y, hx+x, hx-x, hy+y, hy-y}.
// Variant "direct": one node per thread, every side read from memory.
// Variants "vector tile" (below): V adjacent nodes per thread.  All call
// neq_core with the same operands and give identical results.
// ---------------------------------------------------------------------------

template <typename NeqT>
__device__ __forceinline__ void neq_direct_node(const Lattice &L, const void *__restrict__ srcv,
                                                void *__restrict__ dstv, float einc, int i, int j)
{
    const size_t P = L.plane;
    const float *F = reinterpret_cast<const float *>(srcv);
    const NeqT *N = reinterpret_cast<const NeqT *>(F + 3 * P);
    float *DF = reinterpret_cast<float *>(dstv);
    NeqT *DN = reinterpret_cast<NeqT *>(DF + 3 * P);
    const size_t cf = at(i, j, L.sf), cn = at(i, j, L.sn);
    uint8_t m;
    float inv_eps, eps_rest;
    Side l{}, r{}, b{}, t{}, lo{}, hi{};
    node_setup(L, F, N, i, j, cf, cn, m, inv_eps, eps_rest, l, r);
    const NodeData o = load_node(F, N, P, cf, cn);
    NodeData out;
    if (j == L.ny) {
        neq_core<true>(L, i, j, m, coef_of(L, inv_eps, eps_rest), o, l, r, b, t, lo, hi, einc, out);
    } else {
        if (j > 0) b = load_side(F, N, P, cf - L.sf, cn - L.sn, N_EPY, N_HYPY);
        if (j < L.ny - 1) t = load_side(F, N, P, cf + L.sf, cn + L.sn, N_EMY, N_HYMY);
        load_incident_sides(L, F, N, i, j, lo, hi);
        neq_core<false>(L, i, j, m, coef_of(L, inv_eps, eps_rest), o, l, r, b, t, lo, hi, einc, out);
    }
    store_node(DF, DN, P, cf, cn, out, L.stream_stores);
}

template <typename NeqT>
__global__ __launch_bounds__(BX *BY) void k_step_neq(Lattice L, const void *__restrict__ srcv,
                                                      void *__restrict__ dstv, float einc)
{
    int tx, ty;
    block_tile(L, tx, ty);
    const int i = tx * BX + threadIdx.x;
    const int j = ty * BY + threadIdx.y;
    if (i >= L.nx || j > L.ny) return;
    neq_direct_node<NeqT>(L, srcv, dstv, einc, i, j);
}

// ---------------------------------------------------------------------------
// V-wide row access: each thread of the vector variants owns V adjacent
// nodes of a row and moves every plane with one V-wide load or store.
// ---------------------------------------------------------------------------

template <typename T, int V> struct VecOf;
template <> struct VecOf<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct VecOf<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VecOf<__bf16, 2> { typedef __bf16 __attribute__((ext_vector_type(2))) type; };
template <> struct VecOf<__bf16, 4> { typedef __bf16 __attribute__((ext_vector_type(4))) type; };
template <int V> struct MaskVec;
template <> struct MaskVec<1> { typedef unsigned char type; };
template <> struct MaskVec<2> { typedef unsigned short type; };
template <> struct MaskVec<4> { typedef unsigned int type; };

template <typename T, int V>
__device__ __forceinline__ void vload(const T *p, float (&out)[V])
{
    if constexpr (V == 1) {
        out[0] = (float)*p;
    } else {
        const typename VecOf<T, V>::type v = *reinterpret_cast<const typename VecOf<T, V>::type *>(p);
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = (float)v[k];
    }
}

template <typename T, int V>
__device__ __forceinline__ void vstore(T *p, const float (&in)[V], bool stream)
{
    if constexpr (V == 1) {
        put(p, (T)in[0], stream);
    } else {
        typename VecOf<T, V>::type v;
#pragma unroll
        for (int k = 0; k < V; ++k) v[k] = (T)in[k];
        put(reinterpret_cast<typename VecOf<T, V>::type *>(p), v, stream);
    }
}

template <int V>
struct RowData {
    float ez[V], hx[V], hy[V];
    float n[8][V];
};


template <typename NeqT, int V>
__device__ __forceinline__ void load_row(const float *F, const NeqT *N, size_t P, size_t cf, size_t cn, RowData<V> &r)
{
    vload<float, V>(F + cf, r.ez);
    vload<float, V>(F + P + cf, r.hx);
    vload<float, V>(F + 2 * P + cf, r.hy);
#pragma unroll
    for (int q = 0; q < 8; ++q) vload<NeqT, V>(N + q * P + cn, r.n[q]);
}

// Row data at columns col .. col + V - 1 of the lattice row that starts at
// Fr (its field planes, then its deviation planes): a wave-uniform row base
// plus 32-bit offsets that stay the same from row to row.
template <typename NeqT> __device__ __forceinline__ unsigned f_off(unsigned P, int q, unsigned col)
{
    return (q * P + col) * 4u;
}
template <typename NeqT> __device__ __forceinline__ unsigned n_off(unsigned P, int q, unsigned col)
{
    return 12u * P + (q * P + col) * (unsigned)sizeof(NeqT);
}
template <typename T> __device__ __forceinline__ const T *byte_at(const void *base, unsigned off)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T> __device__ __forceinline__ T *byte_at(void *base, unsigned off)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}

template <typename NeqT, int V>
__device__ __forceinline__ void load_row_at(const float *Fr, unsigned P, unsigned col, RowData<V> &r)
{
    vload<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 0, col)), r.ez);
    vload<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 1, col)), r.hx);
    vload<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 2, col)), r.hy);
#pragma unroll
    for (int q = 0; q < 8; ++q) vload<NeqT, V>(byte_at<NeqT>(Fr, n_off<NeqT>(P, q, col)), r.n[q]);
}

template <int V>
__device__ __forceinline__ void zero_row(RowData<V> &r)
{
#pragma unroll
    for (int k = 0; k < V; ++k) {
        r.ez[k] = r.hx[k] = r.hy[k] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) r.n[q][k] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Variant "vector tile": one shot per thread like the direct variant, but
// each thread owns V adjacent nodes of one row: every plane moves with one
// V-wide load or store, the x-neighbours come from the adjacent lanes (the
// wavefront's edge lanes read theirs from memory) and the rows above and
// below are read V-wide.  Blocks are 64 lanes x 4 rows.
// ---------------------------------------------------------------------------

template <typename NeqT, int V>
__device__ __forceinline__ void neq_vtile_row(const Lattice &L, const void *__restrict__ srcv, void *__restrict__ dstv,
                                              float einc, int col, int j)
{
    const size_t P = L.plane;
    const float *F = reinterpret_cast<const float *>(srcv);
    const NeqT *N = reinterpret_cast<const NeqT *>(F + 3 * P);
    float *DF = reinterpret_cast<float *>(dstv);
    NeqT *DN = reinterpret_cast<NeqT *>(DF + 3 * P);
    const int i0 = col * V;
    const int lane = threadIdx.x & 63;
    const bool active = i0 < L.nx && j <= L.ny;
    RowData<V> cur;
    zero_row(cur);
    const size_t cf = at(i0, j, L.sf), cn = at(i0, j, L.sn);
    if (active) load_row<NeqT, V>(F, N, P, cf, cn, cur);
    // x-neighbours across lanes (every lane of the wavefront takes part)
    Side xl, xr;
    xl.ez = from_left(cur.ez[V - 1]);
    xl.hx = from_left(cur.hx[V - 1]);
    xl.hy = from_left(cur.hy[V - 1]);
    xl.na = from_left(cur.n[N_EPX][V - 1]);
    xl.nb = from_left(cur.n[N_HXPX][V - 1]);
    xr.ez = from_right(cur.ez[0]);
    xr.hx = from_right(cur.hx[0]);
    xr.hy = from_right(cur.hy[0]);
    xr.na = from_right(cur.n[N_EMX][0]);
    xr.nb = from_right(cur.n[N_HXMX][0]);
    if (!active) return;
    if (j == L.ny) {
        // companion row: per node, as in the other variants
        for (int v = 0; v < V; ++v)
            if (i0 + v < L.nx) neq_direct_node<NeqT>(L, srcv, dstv, einc, i0 + v, L.ny);
        return;
    }
    if (lane == 0 && i0 > 0) xl = load_side(F, N, P, cf - 1, cn - 1, N_EPX, N_HXPX);
    if (lane == 63 && i0 + V < L.nx) xr = load_side(F, N, P, cf + V, cn + V, N_EMX, N_HXMX);
    // rows below and above, V-wide
    float bz[V], bhx[V], bhy[V], bna[V], bnb[V], tz[V], thx[V], thy[V], tna[V], tnb[V];
#pragma unroll
    for (int v = 0; v < V; ++v) bz[v] = bhx[v] = bhy[v] = bna[v] = bnb[v] = tz[v] = thx[v] = thy[v] = tna[v] = tnb[v] = 0.0f;
    if (j > 0) {
        const size_t bf = cf - L.sf, bn = cn - L.sn;
        vload<float, V>(F + bf, bz);
        vload<float, V>(F + P + bf, bhx);
        vload<float, V>(F + 2 * P + bf, bhy);
        vload<NeqT, V>(N + N_EPY * P + bn, bna);
        vload<NeqT, V>(N + N_HYPY * P + bn, bnb);
    }
    if (j + 1 < L.ny) {
        const size_t tf = cf + L.sf, tn = cn + L.sn;
        vload<float, V>(F + tf, tz);
        vload<float, V>(F + P + tf, thx);
        vload<float, V>(F + 2 * P + tf, thy);
        vload<NeqT, V>(N + N_EMY * P + tn, tna);
        vload<NeqT, V>(N + N_HYMY * P + tn, tnb);
    }
    const typename MaskVec<V>::type mv = *reinterpret_cast<const typename MaskVec<V>::type *>(L.mask + node(L, i0, j));
    RowData<V> out;
    zero_row(out);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        const uint8_t m = (uint8_t)(mv >> (8 * v));
        const int mat = m & 3;
        if (i >= L.nx) continue;
        const float inv_eps = mat_inv_eps_f(L, mat);
        const float eps_rest = mat_eps_rest_f(L, mat);
        NodeData o;
        o.ez = cur.ez[v];
        o.hx = cur.hx[v];
        o.hy = cur.hy[v];
#pragma unroll
        for (int q = 0; q < 8; ++q) o.n[q] = cur.n[q][v];
        const Side l = v == 0 ? xl : Side{cur.ez[v - 1], cur.hx[v - 1], cur.hy[v - 1], cur.n[N_EPX][v - 1], cur.n[N_HXPX][v - 1]};
        const Side r = v == V - 1 ? xr : Side{cur.ez[v + 1], cur.hx[v + 1], cur.hy[v + 1], cur.n[N_EMX][v + 1], cur.n[N_HXMX][v + 1]};
        const Side b{bz[v], bhx[v], bhy[v], bna[v], bnb[v]};
        const Side t{tz[v], thx[v], thy[v], tna[v], tnb[v]};
        Side lo{}, hi{};
        load_incident_sides(L, F, N, i, j, lo, hi);
        NodeData res;
        neq_core<false>(L, i, j, m, coef_of(L, inv_eps, eps_rest), o, l, r, b, t, lo, hi, einc, res);
        out.ez[v] = res.ez;
        out.hx[v] = res.hx;
        out.hy[v] = res.hy;
#pragma unroll
        for (int q = 0; q < 8; ++q) out.n[q][v] = res.n[q];
    }
    vstore<float, V>(DF + cf, out.ez, L.stream_stores);
    vstore<float, V>(DF + P + cf, out.hx, L.stream_stores);
    vstore<float, V>(DF + 2 * P + cf, out.hy, L.stream_stores);
#pragma unroll
    for (int q = 0; q < 8; ++q) vstore<NeqT, V>(DN + q * P + cn, out.n[q], L.stream_stores);
}

template <typename NeqT, int V, int CX, int R>
__global__ __launch_bounds__(CX *R) void k_step_neq_vtile(Lattice L, const void *__restrict__ srcv,
                                                           void *__restrict__ dstv, float einc)
{
    int tx, ty;
    block_tile(L, tx, ty);
    neq_vtile_row<NeqT, V>(L, srcv, dstv, einc, tx * CX + threadIdx.x, ty * R + threadIdx.y);
}


// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking).  The state at n is read once and
// the state at n + 2 written once, so a launch moves the bytes of one step
// for two lattice updates.
//
// One wavefront is one independent work item: a strip of 64 V columns (V
// adjacent nodes per lane) and H output rows.  Step n -> n + 1 is taken on
// the rows j0 - 1 .. j0 + H and on every column of the strip; step
// n + 1 -> n + 2 on rows j0 .. j0 + H - 1 and on all but HX columns at each
// side, whose intermediate values lack an x-neighbour.  Strips therefore
// overlap by 2 HX columns and rows are re-read at segment seams (from L2).
// The wavefront sweeps up the rows keeping, in registers, three rows at n
// (one more in flight) and three at n + 1; x-neighbours come from the
// adjacent lanes.  Both updates call neq_core with the operands the one-step
// kernels give it, and the intermediate deviations are rounded to the
// storage type as a store would: results equal two one-step launches bit for
// bit.  The companion row is stepped alongside where rows 0 or ny - 1 need
// it; the wavefronts of the bottom segment store it.
// ---------------------------------------------------------------------------

template <typename NeqT> __device__ __forceinline__ float rt(float x) { return (float)(NeqT)x; }

// What the rows next to a row pull from it: per node, the post-collision
// pair (e, h) it sends up (+y: N_{e+y}, N_{hy+y}) or down (-y: N_{e-y},
// N_{hy-y}), computed once per row instead of per pulling node.
template <int V>
struct SideRow {
    float e[V], h[V];
};

// qa / qb: N_EPY, N_HYPY for the pair sent up; N_EMY, N_HYMY for the pair
// sent down (compile-time constants at every call).
template <int V>
__device__ __forceinline__ SideRow<V> side_of(const RowData<V> &r, int qa, int qb)
{
#pragma clang fp contract(off)
    SideRow<V> s;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const Side d{r.ez[v], r.hx[v], r.hy[v], r.n[qa][v], r.n[qb][v]};
        s.e[v] = qa == N_EPY ? up_e(d) : down_e(d);
        s.h[v] = qa == N_EPY ? up_h(d) : down_h(d);
    }
    return s;
}

// Companion-row pairs rows 0 and ny - 1 pull from: lo = sent up, hi = sent down.
template <int V>
struct StripSides {
    SideRow<V> lo, hi;
};

// One row's update from its own data (row r), the pairs the rows below and
// above send it, the x-neighbours across lanes, and the companion row.
// Every node of the row is updated without branching on its kind: for nodes
// outside the domain (padding, rows or columns beyond its edges) the result
// is a finite value that no valid node ever reads -- a valid node next to
// such a node takes an edge rule instead -- and mask_row writes zeros for
// the padding.
// Per-node material coefficients of a row (scaled as stored: 1 / (6 eps) and
// 6 (eps - 2/3)); the companion row is vacuum.
template <int V, bool STRIP>
__device__ __forceinline__ void row_coefs(const Lattice &L, typename MaskVec<V>::type mv, float (&ie)[V],
                                          float (&er)[V])
{
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ie[v] = SIXTH;  // vacuum
        er[v] = 2.0f;
        if (!STRIP) {
            const int mat = (int)((mv >> (8 * v)) & 3);
            ie[v] = mat_inv_eps_f(L, mat);
            er[v] = mat_eps_rest_f(L, mat);
        }
    }
}

// One row's update with its material coefficients given (a sweep that
// updates the same row at several levels picks them once).
template <typename NeqT, int V, bool STRIP, int TEM = 2>
__device__ __forceinline__ void row_update_k(const Lattice &L, int i0, int r, typename MaskVec<V>::type mv,
                                             const float (&ie)[V], const float (&er)[V], const RowData<V> &cur,
                                             const SideRow<V> &below, const SideRow<V> &above,
                                             const StripSides<V> &inc, float einc, RowData<V> &out)
{
#pragma clang fp contract(off)
    // the pairs each node sends east (+x) and west (-x)
    float ee[V], eh[V], we[V], wh[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ee[v] = (cur.ez[v] - cur.hy[v]) - cur.n[N_EPX][v];
        eh[v] = cur.hx[v] - cur.n[N_HXPX][v];
        we[v] = (cur.ez[v] + cur.hy[v]) - cur.n[N_EMX][v];
        wh[v] = cur.hx[v] - cur.n[N_HXMX][v];
    }
    const float xl_e = from_left(ee[V - 1]), xl_h = from_left(eh[V - 1]);
    const float xr_e = from_right(we[0]), xr_h = from_right(wh[0]);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        const uint8_t m = STRIP ? (uint8_t)0 : (uint8_t)(mv >> (8 * v));
        NodeData o;
        o.ez = cur.ez[v];
        o.hx = cur.hx[v];
        o.hy = cur.hy[v];
#pragma unroll
        for (int q = 0; q < 8; ++q) o.n[q] = cur.n[q][v];
        const float e_px = v == 0 ? xl_e : ee[v - 1], hx_px = v == 0 ? xl_h : eh[v - 1];
        const float e_mx = v == V - 1 ? xr_e : we[v + 1], hx_mx = v == V - 1 ? xr_h : wh[v + 1];
        NodeData res;
        neq_pulled<STRIP>(L, i, r, m, coef_pick<TEM>(L, ie[v], er[v]), o, e_px, hx_px, e_mx, hx_mx, below.e[v], below.h[v],
                          above.e[v], above.h[v], Pair{inc.lo.e[v], inc.lo.h[v]}, Pair{inc.hi.e[v], inc.hi.h[v]}, einc,
                          res);
        out.ez[v] = res.ez;
        out.hx[v] = res.hx;
        out.hy[v] = res.hy;
#pragma unroll
        for (int q = 0; q < 8; ++q) out.n[q][v] = res.n[q];
    }
}

// One row's update from its own data (row r), the pairs the rows below and
// above send it, the x-neighbours across lanes, and the companion row.
// Every node of the row is updated without branching on its kind: for nodes
// outside the domain (padding, rows or columns beyond its edges) the result
// is a finite value that no valid node ever reads -- a valid node next to
// such a node takes an edge rule instead -- and mask_row writes zeros for
// the padding.
template <typename NeqT, int V, bool STRIP>
__device__ __forceinline__ void row_update(const Lattice &L, int i0, int r, typename MaskVec<V>::type mv,
                                           const RowData<V> &cur, const SideRow<V> &below, const SideRow<V> &above,
                                           const StripSides<V> &inc, float einc, RowData<V> &out)
{
    float ie[V], er[V];
    row_coefs<V, STRIP>(L, mv, ie, er);
    row_update_k<NeqT, V, STRIP>(L, i0, r, mv, ie, er, cur, below, above, inc, einc, out);
}

template <typename NeqT, int V>
__device__ __forceinline__ void round_row(RowData<V> &r)
{
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int v = 0; v < V; ++v) r.n[q][v] = rt<NeqT>(r.n[q][v]);
}

// Zeros for the padding past nx, as the one-step kernels leave it.
template <int V>
__device__ __forceinline__ void mask_row(const Lattice &L, int i0, RowData<V> &o)
{
    bool all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) all = all && i0 + v < L.nx;
    // only the wavefronts at the right edge hold padding: the others skip
    // the selects
    if (__builtin_amdgcn_ballot_w64(!all) == 0) return;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const bool keep = i0 + v < L.nx;
        o.ez[v] = keep ? o.ez[v] : 0.0f;
        o.hx[v] = keep ? o.hx[v] : 0.0f;
        o.hy[v] = keep ? o.hy[v] : 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) o.n[q][v] = keep ? o.n[q][v] : 0.0f;
    }
}

template <typename NeqT, int V>
__device__ __forceinline__ void store_row_at(float *Fr, unsigned P, unsigned col, const RowData<V> &o, bool stream)
{
    vstore<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 0, col)), o.ez, stream);
    vstore<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 1, col)), o.hx, stream);
    vstore<float, V>(byte_at<float>(Fr, f_off<NeqT>(P, 2, col)), o.hy, stream);
#pragma unroll
    for (int q = 0; q < 8; ++q) vstore<NeqT, V>(byte_at<NeqT>(Fr, n_off<NeqT>(P, q, col)), o.n[q], stream);
}

// A wavefront covers 64 V columns: HX halo columns at each side (at least
// the 2 that two updates need; more keep the output strip aligned to 64
// bytes, which matters when the state streams to HBM) and 64 V - 2 HX
// output columns.
template <int V, int HX> constexpr int two_step_width() { return 64 * V - 2 * HX; }

constexpr int TWO_STEP_WAVES = 4;  // independent wavefronts per block

// One wavefront's share of a two-step launch: strip sx, row segment sy.
// With `one`, only the first step is taken and its result stored (a solve
// with a single step left).
template <typename NeqT, int V, int H, int HX, int LA>
__device__ __forceinline__ void two_step_wave(const Lattice &L, const void *__restrict__ srcv,
                                              void *__restrict__ dstv, float einc0, float einc1,
                                              float *__restrict__ mid, int sx, int sy, bool one)
{
    constexpr int OW = two_step_width<V, HX>();
    static_assert(HX >= 2 && HX % V == 0 && OW > 0, "two-step strip shape");
    typedef typename MaskVec<V>::type MaskT;
    const int x0 = sx * OW, j0 = sy * H;
    const int lane = threadIdx.x;
    const int i0 = x0 - HX + V * lane;
    const bool act = i0 >= 0 && i0 < L.nx;
    const bool out_lane = act && lane >= HX / V && lane < (HX + OW) / V;

    const size_t P = L.plane;
    const float *F = reinterpret_cast<const float *>(srcv);
    const NeqT *N = reinterpret_cast<const NeqT *>(F + 3 * P);
    float *DF = reinterpret_cast<float *>(dstv);
    NeqT *DN = reinterpret_cast<NeqT *>(DF + 3 * P);
    // Rows are loaded without a branch, from a clamped (always valid)
    // address, so the look-ahead loads stay in straight-line code ahead of
    // the arithmetic.  What a lane loads for a row or column outside the
    // domain is never used: row_update skips such nodes, and domain-edge
    // nodes take their edge rules instead of the outside neighbour.
    // Addresses: a wave-uniform row base plus a 32-bit lane offset.
    const unsigned Pu = (unsigned)P;
    const unsigned ic = (unsigned)(min(max(i0, 0), L.nx - 1) / V * V);
    auto load = [&](int r, RowData<V> &d, MaskT &m) {
        const int rc = min(max(r, 0), L.ny - 1);
        load_row_at<NeqT, V>(F + (size_t)rc * L.sf, Pu, ic, d);
        m = *byte_at<MaskT>(L.mask + (size_t)rc * L.pitch, ic);
    };

    // companion row at n and n + 1 where rows 0 or ny - 1 are updated here
    StripSides<V> s0{}, s1{};
    if (j0 <= 1 || j0 + H >= L.ny - 1) {
        RowData<V> c0, c1;
        zero_row(c0);
        load_row_at<NeqT, V>(F + (size_t)L.ny * L.sf, Pu, ic, c0);
        row_update<NeqT, V, true>(L, i0, L.ny, 0, c0, SideRow<V>{}, SideRow<V>{}, StripSides<V>{}, einc0, c1);
        round_row<NeqT, V>(c1);
        if (one && j0 == 0) {
            RowData<V> c = c1;
            mask_row<V>(L, i0, c);
            if (out_lane) store_row_at<NeqT, V>(DF + (size_t)L.ny * L.sf, Pu, (unsigned)i0, c, L.stream_stores);
        }
        s0.lo = side_of(c0, N_EPY, N_HYPY);
        s0.hi = side_of(c0, N_EMY, N_HYMY);
        s1.lo = side_of(c1, N_EPY, N_HYPY);
        s1.hi = side_of(c1, N_EMY, N_HYMY);
        if (!one && j0 == 0) {
            RowData<V> c2;
            row_update<NeqT, V, true>(L, i0, L.ny, 0, c1, SideRow<V>{}, SideRow<V>{}, StripSides<V>{}, einc1, c2);
            mask_row<V>(L, i0, c2);
            if (out_lane)
                store_row_at<NeqT, V>(DF + (size_t)L.ny * L.sf, Pu, (unsigned)i0, c2, L.stream_stores);
        }
    }

    // The sweep.  Consecutive row segments run in opposite directions, so the
    // two segments next to a seam read its rows at the same moment (both at
    // the start or both at the end of their sweeps) and the second read hits
    // in L2.  DIR = +1 walks up the rows, -1 down; "behind" is the row the
    // sweep came from, "ahead" the row it goes to.
    auto sweep = [&](auto dir_tag) {
        constexpr int DIR = decltype(dir_tag)::value;
        // sides of the rows below / above a node, by the populations they feed
        constexpr int BQA = DIR > 0 ? N_EPY : N_EMY, BQB = DIR > 0 ? N_HYPY : N_HYMY;  // behind
        constexpr int AQA = DIR > 0 ? N_EMY : N_EPY, AQB = DIR > 0 ? N_HYMY : N_HYPY;  // ahead
        const int first = DIR > 0 ? j0 - 1 : j0 + H;  // first row of step n -> n + 1
        // rows at n: behind (side), cur, ahead, and the rows in flight (LA of
        // them: the load of a row is issued LA iterations before its first
        // use, hiding that much more latency); rows at n + 1: behind (side), cur
        RowData<V> a_cur, a_ahead, a_pre, tmp;
        MaskT m_cur, m_ahead, m_pre = 0, m_prev = 0, m_dummy;
        float ie_prev[V], er_prev[V];  // coefficients of the row behind (m_prev)
#pragma unroll
        for (int v = 0; v < V; ++v) ie_prev[v] = er_prev[v] = 0.0f;
        load(first - DIR, tmp, m_dummy);
        SideRow<V> a_behind = side_of(tmp, BQA, BQB);
        load(first, a_cur, m_cur);
        load(first + DIR, a_ahead, m_ahead);
        if constexpr (LA == 2) load(first + 2 * DIR, a_pre, m_pre);
        else zero_row(a_pre);
        SideRow<V> b_behind{};
        RowData<V> b_cur;
        zero_row(b_cur);
#pragma unroll
        for (int k = 0; k < H + 2; ++k) {
            const int r1 = first + DIR * k;
            RowData<V> a_next;
            MaskT m_next;
            // the last row a step-1 row needs lies one past the segment's halo
            if constexpr (LA == 2) {
                RowData<V> a_far;
                MaskT m_far;
                if (k + 1 <= H) load(r1 + 3 * DIR, a_far, m_far);
                else { a_far = a_pre; m_far = m_pre; }
                a_next = a_pre;
                m_next = m_pre;
                a_pre = a_far;
                m_pre = m_far;
            } else {
                if (k <= H) load(r1 + 2 * DIR, a_next, m_next);
                else { a_next = a_ahead; m_next = m_ahead; }
            }
            // keep the look-ahead loads here, ahead of this row's arithmetic
            // (the scheduler would otherwise sink them next to their first use)
            __builtin_amdgcn_sched_barrier(0);
            // step n -> n + 1 on row r1
            RowData<V> b_new;
            const SideRow<V> a_side = side_of(a_ahead, AQA, AQB);
            float ie[V], er[V];  // the row's material coefficients, reused by the second step
            row_coefs<V, false>(L, m_cur, ie, er);
            row_update_k<NeqT, V, false>(L, i0, r1, m_cur, ie, er, a_cur, DIR > 0 ? a_behind : a_side,
                                         DIR > 0 ? a_side : a_behind, s0, einc0, b_new);
            round_row<NeqT, V>(b_new);
            if (one) {
                // a single step: this row's result is the new state
                if (out_lane && r1 >= j0 && r1 < j0 + H && r1 < L.ny) {
                    RowData<V> o = b_new;
                    mask_row<V>(L, i0, o);
                    store_row_at<NeqT, V>(DF + (size_t)r1 * L.sf, Pu, (unsigned)i0, o, L.stream_stores);
                }
            }
            // fields at n + 1 of the contour-stencil nodes of this segment's rows
            if (mid && out_lane && r1 >= j0 && r1 < j0 + H && r1 < L.ny) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if ((m_cur >> (8 * v)) & MASK_CONTOUR) {
                        float *f = mid + (size_t)r1 * 3 * P + i0 + v;
                        f[0] = b_new.ez[v];
                        f[P] = b_new.hx[v];
                        f[2 * P] = b_new.hy[v];
                    }
            }
            // step n + 1 -> n + 2 on the row behind r1
            if (!one && k >= 2) {
                const int r2 = r1 - DIR;
                RowData<V> o;
                const SideRow<V> b_side = side_of(b_new, AQA, AQB);
                row_update_k<NeqT, V, false>(L, i0, r2, m_prev, ie_prev, er_prev, b_cur,
                                             DIR > 0 ? b_behind : b_side, DIR > 0 ? b_side : b_behind, s1, einc1, o);
                mask_row<V>(L, i0, o);
                if (out_lane && r2 < L.ny)
                    store_row_at<NeqT, V>(DF + (size_t)r2 * L.sf, Pu, (unsigned)i0, o, L.stream_stores);
            }
            b_behind = side_of(b_cur, BQA, BQB);
            b_cur = b_new;
            m_prev = m_cur;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ie_prev[v] = ie[v];
                er_prev[v] = er[v];
            }
            a_behind = side_of(a_cur, BQA, BQB);
            a_cur = a_ahead;
            m_cur = m_ahead;
            a_ahead = a_next;
            m_ahead = m_next;
        }
    };
    if (sy & 1) sweep(std::integral_constant<int, -1>{});
    else sweep(std::integral_constant<int, 1>{});
}

template <typename NeqT, int V, int H, int HX, int LA>
__global__ __launch_bounds__(64 * TWO_STEP_WAVES) void k_step2_neq(Lattice L, const void *__restrict__ srcv,
                                                                    void *__restrict__ dstv, float einc0, float einc1,
                                                                    float *__restrict__ mid, int nsx, int nsy)
{
    // Work order.  A cache-resident state: the segments of one strip follow
    // each other and each XCD takes a contiguous range (the seam rows that
    // neighbouring segments share stay in one L2).  A state streamed from
    // HBM: the strips of one band of rows run side by side, so the rows in
    // flight are whole lattice rows (DRAM page locality).
    const int nb = gridDim.x;
    const int b = L.stream_stores ? (int)blockIdx.x : xcd_tile(blockIdx.x, nb);
    // wave-uniform work item (held in scalar registers)
    const int w = __builtin_amdgcn_readfirstlane(b * TWO_STEP_WAVES + (int)threadIdx.y);
    if (w >= nsx * nsy) return;  // whole wavefront
    const int sx = L.stream_stores ? w % nsx : w / nsy, sy = L.stream_stores ? w / nsx : w % nsy;
    two_step_wave<NeqT, V, H, HX, LA>(L, srcv, dstv, einc0, einc1, mid, sx, sy, false);
}

// A two-step solve takes a multi-step launch while mdepth more levels remain
// (inside the averaging window too: the launch keeps its intermediate levels'
// contour fields and a batched contour launch accumulates the levels).
__device__ __forceinline__ bool multi_mode(const SolveDesc &d, int64_t n)
{
    return d.mdepth > 0 && n + d.mdepth <= d.steps;
}

// Batched two-step launch: wavefront w takes items[w] (slot, strip, row
// segment) of a resident solve at that solve's own step n.
template <typename NeqT, int V, int H, int HX, int LA>
__global__ __launch_bounds__(64 * TWO_STEP_WAVES) void k_step2_neq_batch(SolveDesc *__restrict__ D,
                                                                          const Tile *__restrict__ items, int nitems,
                                                                          int remap)
{
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(b * TWO_STEP_WAVES + (int)threadIdx.y);
    if (w >= nitems) return;
    const Tile t = items[w];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps || multi_mode(d, n)) return;
    const bool one = d.steps - n == 1;
    // middle-level fields are needed when level n + 1 is averaged and a
    // second step follows
    float *mid = !one && n + 1 > d.steps - d.window ? d.mid : nullptr;
    two_step_wave<NeqT, V, H, HX, LA>(d.L, d.state[d.cur], d.state[d.cur ^ 1], (float)batch_incident(d, n),
                                  one ? 0.0f : (float)batch_incident(d, n + 1), mid, t.tx, t.ty, one);
}

// S steps per launch (temporal blocking, S >= 2): the two-step sweep with S
// levels in flight.
// Level s (1-based) updates row r1 - (s - 1) DIR of the sweep from the three
// level-(s - 1) rows around it, the last of which level s - 1 has just
// produced; intermediate levels are rounded to the storage type as a store
// would round them, so the result equals S single steps bit for bit.  A
// segment of H output rows takes H + 2 (S - 1) level-1 rows, and a strip
// needs at least S halo columns at each side.  With MID (inside the
// averaging window) the fields at n + 1 .. n + S - 1 of the contour-stencil
// nodes of the segment's own rows are written to mid, level after level
// (mid_level floats apart, each 3 planes row-interleaved, row stride 3 pitch).
template <typename NeqT, int V, int H, int HX, int S, bool MID, int TEM = 2>
__device__ __forceinline__ void multi_step_wave(const Lattice &L, const void *__restrict__ srcv,
                                                void *__restrict__ dstv, const float (&einc)[S], float *__restrict__ mid,
                                                size_t mid_level, int sx, int sy)
{
    constexpr int OW = two_step_width<V, HX>();
    static_assert(S >= 2 && HX >= S && HX % V == 0 && OW > 0, "multi-step strip shape");
    typedef typename MaskVec<V>::type MaskT;
    const int x0 = sx * OW, j0 = sy * H;
    const int lane = threadIdx.x;
    const int i0 = x0 - HX + V * lane;
    const bool act = i0 >= 0 && i0 < L.nx;
    const bool out_lane = act && lane >= HX / V && lane < (HX + OW) / V;

    const size_t P = L.plane;
    const float *F = reinterpret_cast<const float *>(srcv);
    float *DF = reinterpret_cast<float *>(dstv);
    const unsigned Pu = (unsigned)P;
    // clamped (always valid) row and column: what a lane loads outside the
    // domain is never used (edge nodes take their edge rules)
    const unsigned ic = (unsigned)(min(max(i0, 0), L.nx - 1) / V * V);
    auto load = [&](int r, RowData<V> &d, MaskT &m) {
        const int rc = min(max(r, 0), L.ny - 1);
        load_row_at<NeqT, V>(F + (size_t)rc * L.sf, Pu, ic, d);
        m = *byte_at<MaskT>(L.mask + (size_t)rc * L.pitch, ic);
    };
    // fields of level `lev` (1 .. S - 1) on row r, at its contour-stencil nodes
    auto keep_mid = [&](int lev, int r, const RowData<V> &d, MaskT m) {
        if constexpr (MID) {
            if (mid && out_lane && r >= j0 && r < j0 + H && r < L.ny) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if ((m >> (8 * v)) & MASK_CONTOUR) {
                        float *f = mid + (size_t)(lev - 1) * mid_level + (size_t)r * 3 * P + i0 + v;
                        f[0] = d.ez[v];
                        f[P] = d.hx[v];
                        f[2 * P] = d.hy[v];
                    }
            }
        }
    };

    // companion row at n .. n + S - 1 where rows 0 or ny - 1 are updated at
    // some level; the segment at the bottom also advances it to n + S.  A
    // segment reaches row 0 or row ny - 1, never both (the caller keeps
    // ny >= H + S), so one side per level is kept: the one row 0 pulls from
    // at the bottom, the one row ny - 1 pulls from at the top.
    SideRow<V> edge[S];
#pragma unroll
    for (int s = 0; s < S; ++s) edge[s] = SideRow<V>{};
    if (j0 <= S - 1 || j0 + H >= L.ny - (S - 1)) {
        const bool bottom = j0 <= S - 1;
        RowData<V> c;
        zero_row(c);
        load_row_at<NeqT, V>(F + (size_t)L.ny * L.sf, Pu, ic, c);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            edge[s] = bottom ? side_of(c, N_EPY, N_HYPY) : side_of(c, N_EMY, N_HYMY);
            if (s == S - 1 && j0 != 0) break;
            RowData<V> c2;
            row_update<NeqT, V, true>(L, i0, L.ny, 0, c, SideRow<V>{}, SideRow<V>{}, StripSides<V>{}, einc[s], c2);
            if (s < S - 1) round_row<NeqT, V>(c2);
            c = c2;
        }
        if (j0 == 0) {
            mask_row<V>(L, i0, c);
            if (out_lane) store_row_at<NeqT, V>(DF + (size_t)L.ny * L.sf, Pu, (unsigned)i0, c, L.stream_stores);
        }
    }

    // consecutive row segments sweep in opposite directions (seam rows are
    // read by both neighbours at the same moment and hit in L2)
    auto sweep = [&](auto dir_tag) {
        constexpr int DIR = decltype(dir_tag)::value;
        constexpr int BQA = DIR > 0 ? N_EPY : N_EMY, BQB = DIR > 0 ? N_HYPY : N_HYMY;  // behind
        constexpr int AQA = DIR > 0 ? N_EMY : N_EPY, AQB = DIR > 0 ? N_HYMY : N_HYPY;  // ahead
        constexpr int K = H + 2 * (S - 1);                                             // level-1 rows
        const int first = DIR > 0 ? j0 - (S - 1) : j0 + H - 1 + (S - 1);
        // level 0 (the state at n): behind (side), cur, ahead; levels 1 .. S - 1:
        // behind (side) and cur, the rows level s + 1 is about to update
        RowData<V> a_cur, a_ahead, tmp;
        MaskT m_ahead, m_dummy;
        MaskT mk[S];  // mk[s]: mask of row r1 - s DIR
        float kie[S][V], ker[S][V];  // its material coefficients (picked at level 1)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            mk[s] = 0;
#pragma unroll
            for (int v = 0; v < V; ++v) kie[s][v] = ker[s][v] = 0.0f;
        }
        load(first - DIR, tmp, m_dummy);
        SideRow<V> a_behind = side_of(tmp, BQA, BQB);
        load(first, a_cur, mk[0]);
        load(first + DIR, a_ahead, m_ahead);
        SideRow<V> lv_behind[S];
        RowData<V> lv_cur[S];
#pragma unroll
        for (int s = 1; s < S; ++s) {
            lv_behind[s] = SideRow<V>{};
            zero_row(lv_cur[s]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int r1 = first + DIR * k;
            RowData<V> a_next;
            MaskT m_next;
            if (k <= K - 2) load(r1 + 2 * DIR, a_next, m_next);
            else {
                a_next = a_ahead;
                m_next = m_ahead;
            }
            __builtin_amdgcn_sched_barrier(0);
            // level 1 on row r1
            RowData<V> nw;
            {
                const SideRow<V> side = side_of(a_ahead, AQA, AQB);
                row_coefs<V, false>(L, mk[0], kie[0], ker[0]);
                row_update_k<NeqT, V, false, TEM>(L, i0, r1, mk[0], kie[0], ker[0], a_cur, DIR > 0 ? a_behind : side,
                                             DIR > 0 ? side : a_behind, StripSides<V>{edge[0], edge[0]}, einc[0], nw);
                round_row<NeqT, V>(nw);
                keep_mid(1, r1, nw, mk[0]);
            }
            // levels 2 .. S on the rows behind; nw is the level-s row just made
#pragma unroll
            for (int s = 1; s < S; ++s) {
                if (k < 2 * (s - 1)) break;  // level s has made no row yet
                RowData<V> o;
                const bool go = k >= 2 * s;
                if (go) {
                    const int rs = r1 - s * DIR;
                    const SideRow<V> side = side_of(nw, AQA, AQB);
                    row_update_k<NeqT, V, false, TEM>(L, i0, rs, mk[s], kie[s], ker[s], lv_cur[s],
                                                 DIR > 0 ? lv_behind[s] : side,
                                               DIR > 0 ? side : lv_behind[s], StripSides<V>{edge[s], edge[s]},
                                               einc[s], o);
                    if (s < S - 1) {
                        round_row<NeqT, V>(o);
                        keep_mid(s + 1, rs, o, mk[s]);
                    } else {
                        mask_row<V>(L, i0, o);
                        if (out_lane && rs < L.ny)
                            store_row_at<NeqT, V>(DF + (size_t)rs * L.sf, Pu, (unsigned)i0, o, L.stream_stores);
                    }
                }
                lv_behind[s] = side_of(lv_cur[s], BQA, BQB);
                lv_cur[s] = nw;
                if (!go) break;
                nw = o;
            }
#pragma unroll
            for (int s = S - 1; s > 0; --s) {
                mk[s] = mk[s - 1];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    kie[s][v] = kie[s - 1][v];
                    ker[s][v] = ker[s - 1][v];
                }
            }
            a_behind = side_of(a_cur, BQA, BQB);
            a_cur = a_ahead;
            mk[0] = m_ahead;
            a_ahead = a_next;
            m_ahead = m_next;
        }
    };
    if (sy & 1) sweep(std::integral_constant<int, -1>{});
    else sweep(std::integral_constant<int, 1>{});
}

// S lattice steps per launch; W: wavefronts per SIMD the register
// allocation must allow (more than the registers want costs spills).
// einc: source values of steps n .. n + S - 1.
template <int S> struct Incident {
    float v[S];
};
template <typename NeqT, int V, int H, int HX, int S, int W, bool MID, int TEM>
__global__ __launch_bounds__(64 * TWO_STEP_WAVES, W) void k_stepm_neq(Lattice L, const void *__restrict__ srcv,
                                                                     void *__restrict__ dstv, Incident<S> einc,
                                                                     float *__restrict__ mid, size_t mid_level,
                                                                     int nsx, int nsy)
{
    // work order as for the two-step launch
    const int nb = gridDim.x;
    const int b = L.stream_stores ? (int)blockIdx.x : xcd_tile(blockIdx.x, nb);
    const int w = __builtin_amdgcn_readfirstlane(b * TWO_STEP_WAVES + (int)threadIdx.y);
    if (w >= nsx * nsy) return;  // whole wavefront
    const int sx = L.stream_stores ? w % nsx : w / nsy, sy = L.stream_stores ? w / nsx : w % nsy;
    multi_step_wave<NeqT, V, H, HX, S, MID, TEM>(L, srcv, dstv, einc.v, mid, mid_level, sx, sy);
}

// Batched multi-step launch: wavefront w takes items[w] of a resident solve
// in multi mode at that solve's own step n.
template <typename NeqT, int V, int H, int HX, int S, int W>
__global__ __launch_bounds__(64 * TWO_STEP_WAVES, W) void k_stepm_neq_batch(SolveDesc *__restrict__ D,
                                                                           const Tile *__restrict__ items, int nitems,
                                                                           int remap)
{
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(b * TWO_STEP_WAVES + (int)threadIdx.y);
    if (w >= nitems) return;
    const Tile t = items[w];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps || d.mdepth != S || !multi_mode(d, n)) return;
    float einc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) einc[k] = (float)batch_incident(d, n + k);
    // intermediate levels' contour fields when one of them is averaged
    float *mid = n + S - 1 > d.steps - d.window ? d.mid : nullptr;
    const size_t mid_level = (size_t)3 * d.L.pitch * d.L.ny;
    multi_step_wave<NeqT, V, H, HX, S, true>(d.L, d.state[d.cur], d.state[d.cur ^ 1], einc, mid, mid_level, t.tx,
                                             t.ty);
}

// ---------------------------------------------------------------------------
// Batched steps: block b works on tiles[b] of solve tiles[b].slot at that
// solve's own step n (finished solves return at once).
// ---------------------------------------------------------------------------

template <int CX, int R>
__global__ __launch_bounds__(CX *R) void k_step_f64_batch(SolveDesc *__restrict__ D, const Tile *__restrict__ tiles,
                                                           int remap)
{
    const Tile t = tiles[batch_tile(D, blockIdx.x, gridDim.x, remap)];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps) return;
    const int i = t.tx * CX + threadIdx.x;
    const int j = t.ty * R + threadIdx.y;
    if (i >= d.L.nx || j > d.L.ny) return;
    const bool in_window = n + 1 > d.steps - d.window;
    f64_node(d.L, (const double *)d.state[d.cur], (double *)d.state[d.cur ^ 1],
             in_window ? d.fields + (size_t)((n + 1) & 1) * d.fields_level : nullptr, batch_incident(d, n), i, j);
}

template <typename NeqT>
__global__ __launch_bounds__(BX *BY) void k_step_neq_batch(SolveDesc *__restrict__ D, const Tile *__restrict__ tiles,
                                                            int remap)
{
    const Tile t = tiles[batch_tile(D, blockIdx.x, gridDim.x, remap)];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps) return;
    const int i = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    if (i >= d.L.nx || j > d.L.ny) return;
    neq_direct_node<NeqT>(d.L, d.state[d.cur], d.state[d.cur ^ 1], (float)batch_incident(d, n), i, j);
}

template <typename NeqT, int V, int CX, int R>
__global__ __launch_bounds__(CX *R) void k_step_neq_vtile_batch(SolveDesc *__restrict__ D, const Tile *__restrict__ tiles,
                                                                 int remap)
{
    const Tile t = tiles[batch_tile(D, blockIdx.x, gridDim.x, remap)];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps) return;
    neq_vtile_row<NeqT, V>(d.L, d.state[d.cur], d.state[d.cur ^ 1], (float)batch_incident(d, n),
                           t.tx * CX + threadIdx.x, t.ty * R + threadIdx.y);
}

__global__ void k_advance(SolveDesc *D, int nslots, int which)
{
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        SolveDesc &d = D[s];
        const int64_t n = d.n;
        if (n >= d.steps) continue;
        if (which == 2) {
            if (!d.two || !multi_mode(d, n)) continue;
            d.n = n + d.mdepth;
        } else {
            if (d.two != which || (which == 1 && multi_mode(d, n))) continue;
            d.n = which ? min(n + 2, d.steps) : n + 1;
        }
        d.cur ^= 1;
    }
}

// ---------------------------------------------------------------------------
// Contour sampling (Sec. II.B): bilinear fields at each sample, time sums of
// Ez^2, Hx^2, Hy^2 and Hx Hy in FP64.  One thread per sample, no atomics.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void contour_sample_f64(const Lattice &L, const double *__restrict__ fld,
                                                   const ContourDev &C, int k)
{
#pragma clang fp contract(off)
    const size_t P = L.plane;
    const size_t c00 = at(C.i0[k], C.j0[k], L.sfld);
    const size_t c10 = c00 + L.sfld;
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

// One level's products at sample k added to the running sums s[4].
__device__ __forceinline__ void contour_add_f32(const Lattice &L, const float *__restrict__ fld, size_t stride,
                                                const ContourDev &C, int k, double (&s)[4])
{
#pragma clang fp contract(off)
    const size_t P = L.plane;
    const size_t c00 = at(C.i0[k], C.j0[k], stride);
    const size_t c10 = c00 + stride;
    const float fx = (float)C.wx[k], fy = (float)C.wy[k];
    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy), w10 = (1.0f - fx) * fy, w11 = fx * fy;
    float v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *p = fld + a * P;
        // stored fields are one sixth of the physical ones
        v[a] = 6.0f * (w00 * p[c00] + w01 * p[c00 + 1] + w10 * p[c10] + w11 * p[c10 + 1]);
    }
    s[0] += (double)(v[0] * v[0]);
    s[1] += (double)(v[1] * v[1]);
    s[2] += (double)(v[2] * v[2]);
    s[3] += (double)(v[1] * v[2]);
}

__device__ __forceinline__ void contour_load(const ContourDev &C, int k, double (&s)[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = C.acc[q * C.n + k];
}

__device__ __forceinline__ void contour_store(const ContourDev &C, int k, const double (&s)[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) C.acc[q * C.n + k] = s[q];
}

// One level's products added to the time sums of sample k (the same
// additions, in the same order, as several levels through contour_add_f32).
__device__ __forceinline__ void contour_sample_f32(const Lattice &L, const float *__restrict__ fld, size_t stride,
                                                   const ContourDev &C, int k)
{
    double s[4];
    contour_load(C, k, s);
    contour_add_f32(L, fld, stride, C, k, s);
    contour_store(C, k, s);
}

__global__ void k_contour_f64(Lattice L, const double *__restrict__ fld, ContourDev C)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n) contour_sample_f64(L, fld, C, k);
}

__global__ void k_contour_f32(Lattice L, const float *__restrict__ fld, ContourDev C)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n) contour_sample_f32(L, fld, L.sfld, C, k);
}

// Two consecutive levels: the middle level of a two-step launch (fields of
// the stencil nodes in mid), then the level it ended on (the state).
__global__ void k_contour2_f32(Lattice L, const float *__restrict__ mid, const float *__restrict__ fld, ContourDev C)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n) {
        double s[4];
        contour_load(C, k, s);
        contour_add_f32(L, mid, 3 * L.plane, C, k, s);
        contour_add_f32(L, fld, L.sfld, C, k, s);
        contour_store(C, k, s);
    }
}

// After a multi-step launch inside the window: levels n + 1 .. n + S - 1 from
// mid (mid_level floats apart), then level n + S from the state, in time order.
__global__ void k_contourm_f32(Lattice L, const float *__restrict__ mid, size_t mid_level, int nmid,
                               const float *__restrict__ fld, ContourDev C)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n) {
        double s[4];
        contour_load(C, k, s);
        for (int m = 0; m < nmid; ++m) contour_add_f32(L, mid + (size_t)m * mid_level, 3 * L.plane, C, k, s);
        contour_add_f32(L, fld, L.sfld, C, k, s);
        contour_store(C, k, s);
    }
}

// Batched contour accumulation: block row s serves solve s when the step it
// just took ends inside its averaging window.
__global__ void k_contour_batch(SolveDesc *__restrict__ D)
{
    const SolveDesc &d = D[blockIdx.y];
    const int64_t n = d.n;
    if (d.two || n >= d.steps || !(n + 1 > d.steps - d.window)) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.C.n) return;
    if (d.precision == 0) contour_sample_f64(d.L, d.fields + (size_t)((n + 1) & 1) * d.fields_level, d.C, k);
    else contour_sample_f32(d.L, reinterpret_cast<const float *>(d.state[d.cur ^ 1]), d.L.sfld, d.C, k);
}

// After a batched two-step launch from level n: level n + 1 (the middle
// fields, or the state when the solve had one step left) and level n + 2,
// each if it lies in the averaging window, in that order.
__global__ void k_contour2_batch(SolveDesc *__restrict__ D)
{
    const SolveDesc &d = D[blockIdx.y];
    const int64_t n = d.n;
    if (!d.two || n >= d.steps || multi_mode(d, n)) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.C.n) return;
    const bool one = d.steps - n == 1;
    if (d.precision == 0) {  // FP64: the field planes of each level, by level parity
        if (n + 1 > d.steps - d.window)
            contour_sample_f64(d.L, d.fields + (size_t)((n + 1) & 1) * d.fields_level, d.C, k);
        if (!one && n + 2 > d.steps - d.window)
            contour_sample_f64(d.L, d.fields + (size_t)((n + 2) & 1) * d.fields_level, d.C, k);
        return;
    }
    const float *next = reinterpret_cast<const float *>(d.state[d.cur ^ 1]);
    if (n + 1 > d.steps - d.window) {
        if (one) contour_sample_f32(d.L, next, d.L.sfld, d.C, k);
        else contour_sample_f32(d.L, d.mid, 3 * d.L.plane, d.C, k);
    }
    if (!one && n + 2 > d.steps - d.window) contour_sample_f32(d.L, next, d.L.sfld, d.C, k);
}

// After a batched multi-step launch from level n (before the advance): the
// averaged levels among n + 1 .. n + S, in time order -- the intermediate
// ones from mid, the last from the state it wrote.
__global__ void k_contourm_batch(SolveDesc *__restrict__ D)
{
    const SolveDesc &d = D[blockIdx.y];
    const int64_t n = d.n;
    if (!d.two || n >= d.steps || !multi_mode(d, n)) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.C.n) return;
    const int64_t w0 = d.steps - d.window;  // levels above w0 are averaged
    if (n + d.mdepth <= w0) return;
    const size_t mid_level = (size_t)3 * d.L.pitch * d.L.ny;
    double s[4];
    contour_load(d.C, k, s);
    for (int l = 1; l < d.mdepth; ++l)
        if (n + l > w0) contour_add_f32(d.L, d.mid + (size_t)(l - 1) * mid_level, 3 * d.L.plane, d.C, k, s);
    contour_add_f32(d.L, reinterpret_cast<const float *>(d.state[d.cur ^ 1]), d.L.sfld, d.C, k, s);
    contour_store(d.C, k, s);
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
// Far field (Sec. II.A).  Single-bin phasors over the last period at the
// contour samples: for each level t, dft += F(t) (cos, sin)(omega t) for the
// bilinear Ez, Hx, Hy and for the incident wave's Ez, Hx, Hy from the
// companion row (row ny) at the sample's x.  Layout [12][n]: (re, im) of
// Ez, Hx, Hy, then of the incident Ez, Hx, Hy.  FP64 arithmetic on the stored
// fields; one thread per sample, no atomics.
// ---------------------------------------------------------------------------

template <typename FT>
__global__ void k_far_dft(Lattice L, const FT *__restrict__ fld, ContourDev C, double *__restrict__ dft, double cw,
                          double sw)
{
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.n) return;
    const size_t P = L.plane;
    const int i0 = C.i0[k];
    const size_t c00 = at(i0, C.j0[k], L.sfld);
    const size_t c10 = c00 + L.sfld;
    const size_t cs = at(i0, L.ny, L.sfld);
    const double fx = C.wx[k], fy = C.wy[k];
    const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy), w10 = (1.0 - fx) * fy, w11 = fx * fy;
    const double fs = field_scale<FT>();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const FT *p = fld + a * P;
        const double v = fs * (w00 * (double)p[c00] + w01 * (double)p[c00 + 1] + w10 * (double)p[c10] +
                               w11 * (double)p[c10 + 1]);
        const double u = fs * ((1.0 - fx) * (double)p[cs] + fx * (double)p[cs + 1]);
        dft[(2 * a) * C.n + k] += v * cw;
        dft[(2 * a + 1) * C.n + k] += v * sw;
        dft[(6 + 2 * a) * C.n + k] += u * cw;
        dft[(7 + 2 * a) * C.n + k] += u * sw;
    }
}

// Near-to-far-field transform of the phasors (scale 2 / T turns the sums into
// amplitudes; scattered = total - incident).  With exp(-j omega t), curl E =
// j k0 H and the outward normal n at r' = rc n:
//   I(phi) = sum_k w [J_z - (n.u) E_z^S] exp(-j k0 u.r'),  J_z = n_x H_y - n_y H_x,
//   |S(phi)|^2 = k0^2 |I|^2 / (8 pi |E^I|^2),  u = (cos phi, sin phi),
// |E^I|^2 the mean incident intensity over the samples, w = 2 pi rc / n.
// One wave per angle (blocks of 64); fixed-order wave reductions.
__global__ __launch_bounds__(64) void k_far_field(ContourDev C, const double *__restrict__ dft, double k0,
                                                  double scale, int nphi, double *__restrict__ s2)
{
    const int a = blockIdx.x;
    const int t = threadIdx.x;
    if (a >= nphi) return;
    const int n = C.n;
    const double phi = 2.0 * M_PI * (double)a / (double)nphi;
    const double ux = cos(phi), uy = sin(phi);
    double ire = 0.0, iim = 0.0, ei2 = 0.0;
    for (int k = t; k < n; k += 64) {
        const double nx = C.nxk[k], ny = C.nyk[k];
        double re[3], im[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            re[q] = scale * (dft[(2 * q) * n + k] - dft[(6 + 2 * q) * n + k]);
            im[q] = scale * (dft[(2 * q + 1) * n + k] - dft[(7 + 2 * q) * n + k]);
        }
        const double ir = scale * dft[6 * n + k], ii = scale * dft[7 * n + k];
        ei2 += ir * ir + ii * ii;
        const double nu = nx * ux + ny * uy;
        const double fre = (nx * re[2] - ny * re[1]) - nu * re[0];
        const double fim = (nx * im[2] - ny * im[1]) - nu * im[0];
        double sp, cp;
        sincos(-k0 * C.rc * nu, &sp, &cp);
        ire += fre * cp - fim * sp;
        iim += fre * sp + fim * cp;
    }
    ire = wave_sum(ire);
    iim = wave_sum(iim);
    ei2 = wave_sum(ei2);
    if (t == 0) {
        const double w = 2.0 * M_PI * C.rc / (double)n;
        ire *= w;
        iim *= w;
        s2[a] = k0 * k0 * (ire * ire + iim * iim) / (8.0 * M_PI * (ei2 / (double)n));
    }
}

// Instantaneous stress integral (Sec. II.B with the fields of one level
// instead of their time average): F~x, F~y, M~z into out[0..2].  One block,
// samples strided over the threads, FP64 sums in a fixed order.  The dual
// TE^z storage needs no change: the stress only holds squares and the
// product of the two in-plane components.
template <typename FT>
__global__ __launch_bounds__(RED_THREADS) void k_force_now(Lattice L, const FT *__restrict__ fld, ContourDev C,
                                                           double f0, double m0, double *out)
{
    __shared__ double part[3][RED_THREADS / 64];
    const int t = threadIdx.x;
    const size_t P = L.plane;
    const double w = 2.0 * M_PI * C.rc / C.n;
    double fx = 0.0, fy = 0.0, tz = 0.0;
    for (int k = t; k < C.n; k += RED_THREADS) {
        const size_t c00 = at(C.i0[k], C.j0[k], L.sfld), c10 = c00 + L.sfld;
        const double ax = C.wx[k], ay = C.wy[k];
        const double w00 = (1.0 - ax) * (1.0 - ay), w01 = ax * (1.0 - ay), w10 = (1.0 - ax) * ay, w11 = ax * ay;
        double v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const FT *p = fld + a * P;
            v[a] = field_scale<FT>() *
                   (w00 * (double)p[c00] + w01 * (double)p[c00 + 1] + w10 * (double)p[c10] + w11 * (double)p[c10 + 1]);
        }
        const double txx = 0.5 * (v[1] * v[1] - v[2] * v[2] - v[0] * v[0]);
        const double tyy = 0.5 * (v[2] * v[2] - v[1] * v[1] - v[0] * v[0]);
        const double txy = v[1] * v[2];
        const double nx = C.nxk[k], ny = C.nyk[k];
        const double tx = txx * nx + txy * ny, ty = txy * nx + tyy * ny;
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
        double s3[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < RED_THREADS / 64; ++b) s3[a] += part[a][b];
        out[0] = s3[0] / f0;
        out[1] = s3[1] / f0;
        out[2] = s3[2] / m0;
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
            const int mat = L.mask[node(L, i, j)] & 3;
            if (mat == MAT_PEC) continue;
            const size_t c = at(i, j, L.sfld);
            const double fs = field_scale<FT>();
            const double ez = fs * fld[c], hx = fs * fld[P + c], hy = fs * fld[2 * P + c];
            if (L.te) s += 0.5 * (ez * ez + mat_eps(L, mat) * (hx * hx + hy * hy));
            else s += 0.5 * (mat_eps(L, mat) * ez * ez + hx * hx + hy * hy);
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
    const size_t c = at(i, j, L.sfld);
    const size_t o = (size_t)j * L.nx + i;
    // TE^z: the dual storage holds (Hz, -Ex, -Ey); report (Hz, Ex, Ey);
    // conductor nodes report zero fields
    const double sxy = L.te ? -1.0 : 1.0;
    const double fs = (L.mask[node(L, i, j)] & 3) == MAT_PEC ? 0.0 : field_scale<FT>();
    ez[o] = fs * (double)fld[c];
    hx[o] = sxy * fs * (double)fld[P + c];
    hy[o] = sxy * fs * (double)fld[2 * P + c];
}

dim3 step_grid(const Lattice &L) { return dim3((L.nx + BX - 1) / BX, (L.ny + 1 + BY - 1) / BY); }

}  // namespace

hipError_t launch_step_neq(int precision, const Lattice &L, const void *src, void *dst, double einc, hipStream_t s,
                           int variant)
{
    const float e = (float)einc;
    auto vtile_grid = [&](int v, int cx, int r) { return dim3((L.nx + cx * v - 1) / (cx * v), (L.ny + 1 + r - 1) / r); };
#define JLB_NEQ_LAUNCH(T)                                                                                                    \
    switch (variant) {                                                                                                       \
    case NEQ_TILE_V2: hipLaunchKernelGGL((k_step_neq_vtile<T, 2, 64, 4>), vtile_grid(2, 64, 4), dim3(64, 4), 0, s, L, src, dst, e); break;     \
    case NEQ_TILE_V4: hipLaunchKernelGGL((k_step_neq_vtile<T, 4, 64, 4>), vtile_grid(4, 64, 4), dim3(64, 4), 0, s, L, src, dst, e); break;     \
    case NEQ_TILE_V2_W256: hipLaunchKernelGGL((k_step_neq_vtile<T, 2, 256, 1>), vtile_grid(2, 256, 1), dim3(256, 1), 0, s, L, src, dst, e); break; \
    case NEQ_TILE_V4_W256: hipLaunchKernelGGL((k_step_neq_vtile<T, 4, 256, 1>), vtile_grid(4, 256, 1), dim3(256, 1), 0, s, L, src, dst, e); break; \
    case NEQ_TILE_V2_W256_R2: hipLaunchKernelGGL((k_step_neq_vtile<T, 2, 256, 2>), vtile_grid(2, 256, 2), dim3(256, 2), 0, s, L, src, dst, e); break; \
    case NEQ_TILE_V4_W256_R2: hipLaunchKernelGGL((k_step_neq_vtile<T, 4, 256, 2>), vtile_grid(4, 256, 2), dim3(256, 2), 0, s, L, src, dst, e); break; \
    default: hipLaunchKernelGGL(k_step_neq<T>, step_grid(L), dim3(BX, BY), 0, s, L, src, dst, e); break;                 \
    }
    if (precision == 1) {
        JLB_NEQ_LAUNCH(float)
    } else {
        JLB_NEQ_LAUNCH(__bf16)
    }
#undef JLB_NEQ_LAUNCH
    return hipGetLastError();
}

// Variant dispatch shared by the single-solve and batched two-step launchers.
template <typename F> static void two_step_dispatch(int variant, F &&go)
{
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using H4 = std::integral_constant<int, 4>;
    using H8 = std::integral_constant<int, 8>;
    using H16 = std::integral_constant<int, 16>;
    using H32 = std::integral_constant<int, 32>;
    using X2 = std::integral_constant<int, 2>;
    using X8 = std::integral_constant<int, 8>;
    using L1 = std::integral_constant<int, 1>;
    using L2 = std::integral_constant<int, 2>;
    switch (variant) {
    case TWO_V1_H8_X2: go(I1{}, H8{}, X2{}, L1{}); break;
    case TWO_V1_H16_X2: go(I1{}, H16{}, X2{}, L1{}); break;
    case TWO_V2_H8_X2: go(I2{}, H8{}, X2{}, L1{}); break;
    case TWO_V2_H16_X2: go(I2{}, H16{}, X2{}, L1{}); break;
    case TWO_V1_H8_X8: go(I1{}, H8{}, X8{}, L1{}); break;
    case TWO_V2_H16_X8: go(I2{}, H16{}, X8{}, L1{}); break;
    case TWO_V2_H32_X8: go(I2{}, H32{}, X8{}, L1{}); break;
    case TWO_V1_H8_X8_LA2: go(I1{}, H8{}, X8{}, L2{}); break;
    case TWO_V1_H4_X8_LA2: go(I1{}, H4{}, X8{}, L2{}); break;
    default: go(I1{}, H16{}, X8{}, L2{}); break;
    }
}

void two_step_shape(int variant, int nx, int ny, int &nsx, int &nsy)
{
    two_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto) {
        constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
        nsx = (nx + two_step_width<V, HX>() - 1) / two_step_width<V, HX>();
        nsy = (ny + H - 1) / H;
    });
}

hipError_t launch_step2_neq(int precision, const Lattice &L, const void *src, void *dst, double einc0, double einc1,
                            float *mid, hipStream_t s, int variant)
{
    const float e0 = (float)einc0, e1 = (float)einc1;
    auto run = [&](auto tag) {
        typedef decltype(tag) T;
        two_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto ltag) {
            constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
            constexpr int LA = decltype(ltag)::value;
            const int nsx = (L.nx + two_step_width<V, HX>() - 1) / two_step_width<V, HX>();
            const int nsy = (L.ny + H - 1) / H;
            const int blocks = (nsx * nsy + TWO_STEP_WAVES - 1) / TWO_STEP_WAVES;
            hipLaunchKernelGGL((k_step2_neq<T, V, H, HX, LA>), dim3(blocks), dim3(64, TWO_STEP_WAVES), 0, s, L, src, dst,
                               e0, e1, mid, nsx, nsy);
        });
    };
    if (precision == 1) run(float{});
    else run(__bf16{});
    return hipGetLastError();
}

hipError_t launch_step2_batch(int precision, int variant, SolveDesc *d, const Tile *items, int nitems, int remap,
                              hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int blocks = (nitems + TWO_STEP_WAVES - 1) / TWO_STEP_WAVES;
    auto run = [&](auto tag) {
        typedef decltype(tag) T;
        two_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto ltag) {
            constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
            constexpr int LA = decltype(ltag)::value;
            hipLaunchKernelGGL((k_step2_neq_batch<T, V, H, HX, LA>), dim3(blocks), dim3(64, TWO_STEP_WAVES), 0, s, d,
                               items, nitems, remap);
        });
    };
    if (precision == 1) run(float{});
    else run(__bf16{});
    return hipGetLastError();
}

// Variant table of the multi-step kernels: depth S, rows H, halo columns HX,
// wavefronts per SIMD W.
template <typename F> static void multi_step_dispatch(int variant, F &&go)
{
    using I1 = std::integral_constant<int, 1>;
    using X4 = std::integral_constant<int, 4>;
    using X8 = std::integral_constant<int, 8>;
    using S3 = std::integral_constant<int, 3>;
    using S4 = std::integral_constant<int, 4>;
    using W2 = std::integral_constant<int, 2>;
    using H10 = std::integral_constant<int, 10>;
    using H12 = std::integral_constant<int, 12>;
    using H16 = std::integral_constant<int, 16>;
    switch (variant) {
    case MULTI_S4_H10_X4: go(I1{}, H10{}, X4{}, S4{}, W2{}); break;
    case MULTI_S4_H12_X4: go(I1{}, H12{}, X4{}, S4{}, W2{}); break;
    case MULTI_S4_H16_X4: go(I1{}, H16{}, X4{}, S4{}, W2{}); break;
    case MULTI_S3_H10_X4: go(I1{}, H10{}, X4{}, S3{}, W2{}); break;
    case MULTI_S3_H12_X4: go(I1{}, H12{}, X4{}, S3{}, W2{}); break;
    case MULTI_S4_H12_X8: go(I1{}, H12{}, X8{}, S4{}, W2{}); break;
    case MULTI_S3_H7_X4: go(I1{}, std::integral_constant<int, 7>{}, X4{}, S3{}, W2{}); break;
    default: go(I1{}, std::integral_constant<int, 8>{}, X4{}, S3{}, W2{}); break;
    }
}

void multi_step_grid(int variant, int nx, int ny, int &nsx, int &nsy)
{
    multi_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto, auto) {
        constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
        nsx = (nx + two_step_width<V, HX>() - 1) / two_step_width<V, HX>();
        nsy = (ny + H - 1) / H;
    });
}

void multi_step_shape(int variant, int &depth, int &rows)
{
    multi_step_dispatch(variant, [&](auto, auto htag, auto, auto stag, auto) {
        rows = decltype(htag)::value;
        depth = decltype(stag)::value;
    });
}

hipError_t launch_stepm_neq(int precision, const Lattice &L, const void *src, void *dst, const double *einc,
                            float *mid, size_t mid_level, hipStream_t s, int variant)
{
    int depth = 0, rows = 0;
    multi_step_shape(variant, depth, rows);
    // a segment must not reach both edge rows (callers check first)
    if (L.ny < rows + depth) return hipErrorInvalidValue;
    auto run = [&](auto tag) {
        typedef decltype(tag) T;
        multi_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto stag, auto wtag) {
            constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
            constexpr int S = decltype(stag)::value, W = decltype(wtag)::value;
            Incident<S> e;
            for (int k = 0; k < S; ++k) e.v[k] = (float)einc[k];
            const int nsx = (L.nx + two_step_width<V, HX>() - 1) / two_step_width<V, HX>();
            const int nsy = (L.ny + H - 1) / H;
            const int blocks = (nsx * nsy + TWO_STEP_WAVES - 1) / TWO_STEP_WAVES;
            // the polarisation as a kernel instance (no per-node choice)
            auto go = [&](auto mtag, auto ptag) {
                constexpr bool MID = decltype(mtag)::value;
                constexpr int TEM = decltype(ptag)::value;
                hipLaunchKernelGGL((k_stepm_neq<T, V, H, HX, S, W, MID, TEM>), dim3(blocks),
                                   dim3(64, TWO_STEP_WAVES), 0, s, L, src, dst, e, MID ? mid : nullptr,
                                   MID ? mid_level : (size_t)0, nsx, nsy);
            };
            using TM = std::integral_constant<int, 0>;
            using TE = std::integral_constant<int, 1>;
            if (mid) {
                if (L.te) go(std::true_type{}, TE{});
                else go(std::true_type{}, TM{});
            } else {
                if (L.te) go(std::false_type{}, TE{});
                else go(std::false_type{}, TM{});
            }
        });
    };
    if (precision == 1) run(float{});
    else run(__bf16{});
    return hipGetLastError();
}

hipError_t launch_stepm_batch(int precision, int variant, SolveDesc *d, const Tile *items, int nitems, int remap,
                              hipStream_t s)
{
    int depth = 0, rows = 0;
    multi_step_shape(variant, depth, rows);
    if (depth != 4) return hipErrorInvalidValue;  // the engine steps in rounds of four
    if (nitems <= 0) return hipSuccess;
    const int blocks = (nitems + TWO_STEP_WAVES - 1) / TWO_STEP_WAVES;
    auto run = [&](auto tag) {
        typedef decltype(tag) T;
        multi_step_dispatch(variant, [&](auto vtag, auto htag, auto xtag, auto stag, auto wtag) {
            constexpr int V = decltype(vtag)::value, H = decltype(htag)::value, HX = decltype(xtag)::value;
            constexpr int S = decltype(stag)::value, W = decltype(wtag)::value;
            // the engine steps in rounds of four
            if constexpr (S == 4)
                hipLaunchKernelGGL((k_stepm_neq_batch<T, V, H, HX, S, W>), dim3(blocks), dim3(64, TWO_STEP_WAVES), 0,
                                   s, d, items, nitems, remap);
        });
    };
    if (precision == 1) run(float{});
    else run(__bf16{});
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

hipError_t launch_contour2(const Lattice &L, const float *mid, const void *state, const ContourDev &C, hipStream_t s)
{
    const int threads = 128;
    const int blocks = (C.n + threads - 1) / threads;
    hipLaunchKernelGGL(k_contour2_f32, dim3(blocks), dim3(threads), 0, s, L, mid, (const float *)state, C);
    return hipGetLastError();
}

hipError_t launch_contourm(const Lattice &L, const float *mid, size_t mid_level, int nmid, const void *state,
                           const ContourDev &C, hipStream_t s)
{
    const int threads = 128;
    const int blocks = (C.n + threads - 1) / threads;
    hipLaunchKernelGGL(k_contourm_f32, dim3(blocks), dim3(threads), 0, s, L, mid, mid_level, nmid,
                       (const float *)state, C);
    return hipGetLastError();
}

hipError_t launch_far_dft(int precision, const Lattice &L, const void *fields, const ContourDev &C, double *dft,
                          double cw, double sw, hipStream_t s)
{
    const int threads = 128, blocks = (C.n + threads - 1) / threads;
    if (precision == 0)
        hipLaunchKernelGGL(k_far_dft<double>, dim3(blocks), dim3(threads), 0, s, L, (const double *)fields, C, dft, cw,
                           sw);
    else
        hipLaunchKernelGGL(k_far_dft<float>, dim3(blocks), dim3(threads), 0, s, L, (const float *)fields, C, dft, cw, sw);
    return hipGetLastError();
}

hipError_t launch_force_now(int precision, const Lattice &L, const void *fields, const ContourDev &C, double f0,
                            double m0, double *out, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_force_now<double>, dim3(1), dim3(RED_THREADS), 0, s, L, (const double *)fields, C, f0, m0,
                           out);
    else
        hipLaunchKernelGGL(k_force_now<float>, dim3(1), dim3(RED_THREADS), 0, s, L, (const float *)fields, C, f0, m0,
                           out);
    return hipGetLastError();
}

hipError_t launch_far_field(const ContourDev &C, const double *dft, double k0, double scale, int nphi, double *s2,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_far_field, dim3(nphi), dim3(64), 0, s, C, dft, k0, scale, nphi, s2);
    return hipGetLastError();
}

hipError_t launch_reduce(const ContourDev &C, double inv_window, double f0, double m0, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, s, C, inv_window, f0, m0, out);
    return hipGetLastError();
}

void tile_shape(int precision, int variant, int &cols, int &rows)
{
    if (precision == 0) {
        cols = variant == F64_W256_R1 || variant == F64_W256_R2 ? 256 : BX;
        rows = variant == F64_W256_R1 ? 1 : variant == F64_W256_R2 ? 2 : 4;
        return;
    }
    if (variant == NEQ_DIRECT || variant < 0 || variant >= NEQ_VARIANTS) {
        cols = BX;
        rows = BY;
        return;
    }
    static const int tv[6] = {2, 4, 2, 4, 2, 4}, tc[6] = {64, 64, 256, 256, 256, 256}, tr[6] = {4, 4, 1, 1, 2, 2};
    cols = tc[variant - NEQ_TILE_V2] * tv[variant - NEQ_TILE_V2];
    rows = tr[variant - NEQ_TILE_V2];
}

hipError_t launch_step_batch(int precision, int variant, SolveDesc *d, const Tile *tiles, int ntiles, int remap,
                             hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (precision == 0) {
        switch (variant) {
        case F64_W256_R1: hipLaunchKernelGGL((k_step_f64_batch<256, 1>), dim3(ntiles), dim3(256, 1), 0, s, d, tiles, remap); break;
        case F64_W256_R2: hipLaunchKernelGGL((k_step_f64_batch<256, 2>), dim3(ntiles), dim3(256, 2), 0, s, d, tiles, remap); break;
        default: hipLaunchKernelGGL((k_step_f64_batch<BX, 4>), dim3(ntiles), dim3(BX, 4), 0, s, d, tiles, remap); break;
        }
        return hipGetLastError();
    }
    const dim3 g(ntiles);
#define JLB_BATCH_LAUNCH(T)                                                                                         \
    switch (variant) {                                                                                              \
    case NEQ_TILE_V2: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 2, 64, 4>), g, dim3(64, 4), 0, s, d, tiles, remap); break;      \
    case NEQ_TILE_V4: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 4, 64, 4>), g, dim3(64, 4), 0, s, d, tiles, remap); break;      \
    case NEQ_TILE_V2_W256: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 2, 256, 1>), g, dim3(256, 1), 0, s, d, tiles, remap); break; \
    case NEQ_TILE_V4_W256: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 4, 256, 1>), g, dim3(256, 1), 0, s, d, tiles, remap); break; \
    case NEQ_TILE_V2_W256_R2: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 2, 256, 2>), g, dim3(256, 2), 0, s, d, tiles, remap); break; \
    case NEQ_TILE_V4_W256_R2: hipLaunchKernelGGL((k_step_neq_vtile_batch<T, 4, 256, 2>), g, dim3(256, 2), 0, s, d, tiles, remap); break; \
    default: hipLaunchKernelGGL(k_step_neq_batch<T>, g, dim3(BX, BY), 0, s, d, tiles, remap); break;                      \
    }
    if (precision == 1) {
        JLB_BATCH_LAUNCH(float)
    } else {
        JLB_BATCH_LAUNCH(__bf16)
    }
#undef JLB_BATCH_LAUNCH
    return hipGetLastError();
}

hipError_t launch_contour_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_contour_batch, dim3((max_nc + 127) / 128, nslots), dim3(128), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_contour2_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_contour2_batch, dim3((max_nc + 127) / 128, nslots), dim3(128), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_contourm_batch(SolveDesc *d, int nslots, int max_nc, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_contourm_batch, dim3((max_nc + 127) / 128, nslots), dim3(128), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_advance(SolveDesc *d, int nslots, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, s, d, nslots, which);
    return hipGetLastError();
}

// Plain copy, one 16-byte element per lane over one grid covering the
// buffer (on this part a one-shot grid outruns grid-stride loops): the
// reference kernel for bandwidth and for calibrating memory-traffic counters.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n16)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) dst[k] = src[k];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16);
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

// ---------------------------------------------------------------------------
// Library-held scratch for callers that cannot allocate device memory
// (jlb_solve_static).  One array per device, zero at load, kept until the
// process ends.  In host code the array's name is only a stand-in: its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is ever handed to kernels or
// copies.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void **ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace jlb
