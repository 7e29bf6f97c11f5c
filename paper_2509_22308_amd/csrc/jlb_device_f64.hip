// gfx950 kernels of the FP64 lattice update (11 populations per node): one
// step per launch, and two steps per launch (temporal blocking).
//
// Arithmetic (arXiv 2509.22308 Sec. III, Eq. (LBGK equation) with the
// equilibria of Eq. (equilibrium distribution functions), tau = 1/2, in the
// reduced 11-population TM^z form; populations
//   0 e_r  1 e_{+x}  2 e_{-x}  3 e_{+y}  4 e_{-y}  5 hx_r  6 hx_{+x}  7 hx_{-x}
//   8 hy_r 9 hy_{+y} 10 hy_{-y}):
// a node gathers the post-collision populations that stream into it (the
// pull, with the edge rules), forms the moments and stores f* = 2 f^eq - f.
// Both kernels call the same collision (f64_collide: reciprocals rounded
// once in place of the divisions) with the same operands and without FMA
// contraction, so a two-step launch equals two one-step launches bit for
// bit.  Conductor nodes (Sec. II, E_z^tot = 0) are updated like the others
// with their electric field set to zero, the limit of infinite permittivity.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "jlb_device_common.h"
#include "jlb_internal.h"

namespace jlb {

namespace {

template <int CX, int R>
__global__ __launch_bounds__(CX *R) void k_step_f64(Lattice L, const double *__restrict__ src,
                                                     double *__restrict__ dst, double *__restrict__ fields, double einc)
{
    int tx, ty;
    block_tile(L, tx, ty);
    const int i = tx * CX + threadIdx.x;
    const int j = ty * R + threadIdx.y;
    if (i >= L.nx || j > L.ny) return;
    f64_node(L, src, dst, fields, einc, i, j);
}

// ---------------------------------------------------------------------------
// One step, two adjacent nodes per thread.  Every plane moves with one
// 16-byte access per lane, half the memory instructions of one node per
// thread.  Of the populations that cross between the two nodes of a lane,
// each node takes its partner's directly; those that cross between lanes
// come from the adjacent lane through DPP wave shifts (two 32-bit halves per
// double), and the wavefront's end lanes load theirs.  Each node gathers its
// pulls and edge rules as f64_node does and takes the same collision, so the
// result equals the one-node kernels' bit for bit.  Whole wavefronts run to
// the end (the shifts need every lane); lanes past the lattice load from a
// clamped address and store nothing.
// ---------------------------------------------------------------------------

typedef double __attribute__((ext_vector_type(2))) Double2;

__device__ __forceinline__ Double2 ld2(const double *p) { return *reinterpret_cast<const Double2 *>(p); }

// Lane k receives lane k - 1's v (from_left) or lane k + 1's (from_right);
// the end lane, which has no such neighbour in the wavefront, receives edge.
__device__ __forceinline__ double shift64(double v, double edge, bool left)
{
    const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
    const int blo = (int)(b & 0xffffffff), bhi = (int)(b >> 32);
    const int elo = (int)(e & 0xffffffff), ehi = (int)(e >> 32);
    int lo, hi;
    if (left) {
        lo = __builtin_amdgcn_update_dpp(elo, blo, 0x138, 0xf, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(ehi, bhi, 0x138, 0xf, 0xf, false);
    } else {
        lo = __builtin_amdgcn_update_dpp(elo, blo, 0x130, 0xf, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(ehi, bhi, 0x130, 0xf, 0xf, false);
    }
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int CX, int R>
__global__ __launch_bounds__(CX *R) void k_step_f64_pair(Lattice L, const double *__restrict__ src,
                                                          double *__restrict__ dst, double *__restrict__ fields,
                                                          double einc)
{
#pragma clang fp contract(off)
    static_assert(CX % 64 == 0, "whole wavefronts along a row");
    int tx, ty;
    block_tile(L, tx, ty);
    const int i = 2 * (tx * CX + (int)threadIdx.x);  // nodes i and i + 1
    const int j = ty * R + (int)threadIdx.y;
    const int lane = (int)threadIdx.x & 63;
    const bool valid = i < L.nx && j <= L.ny;
    const bool second = i + 1 < L.nx;  // node i + 1 is in the lattice
    const int ic = min(i, (L.nx - 1) & ~1), jc = min(j, L.ny);
    const size_t P = L.plane;
    const size_t c = at(ic, jc, L.sf);
    const double keep = 1.0 - OPEN_DELTA;

    // populations 1, 6 (moving +x) and 2, 7 (moving -x) of both nodes: what
    // the x-neighbours pull
    const Double2 p1 = ld2(src + 1 * P + c), p6 = ld2(src + 6 * P + c);
    const Double2 p2 = ld2(src + 2 * P + c), p7 = ld2(src + 7 * P + c);
    // the wavefront's end lanes load the values from beyond it
    double e1 = 0.0, e6 = 0.0, e2 = 0.0, e7 = 0.0;
    if (lane == 0 && ic > 0) { e1 = src[1 * P + c - 1]; e6 = src[6 * P + c - 1]; }
    if (lane == 63 && ic + 2 < L.nx) { e2 = src[2 * P + c + 2]; e7 = src[7 * P + c + 2]; }
    const double l1 = shift64(p1.y, e1, true), l6 = shift64(p6.y, e6, true);    // node i - 1
    const double r2 = shift64(p2.x, e2, false), r7 = shift64(p7.x, e7, false);  // node i + 2

    const Double2 o0 = ld2(src + 0 * P + c), o5 = ld2(src + 5 * P + c), o8 = ld2(src + 8 * P + c);
    double f[2][11];
    double inv_eps[2] = {1.0, 1.0}, eps_rest[2] = {1.0 - 2.0 / 3.0, 1.0 - 2.0 / 3.0};
    bool conductor[2] = {false, false};
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        f[v][0] = v ? o0.y : o0.x;
        f[v][5] = v ? o5.y : o5.x;
        f[v][8] = v ? o8.y : o8.x;
    }
    // +x populations come from the node on the left; node 0 takes the source
    f[0][1] = l1; f[0][6] = l6;
    f[1][1] = p1.x; f[1][6] = p6.x;
    if (ic == 0) { f[0][1] = einc / 3.0; f[0][6] = 0.0; }
    if (jc == L.ny) {
        // incident-wave companion row: vacuum, uniform in y, nothing enters on the right
        const Double2 q3 = ld2(src + 3 * P + c), q4 = ld2(src + 4 * P + c);
        const Double2 q9 = ld2(src + 9 * P + c), q10 = ld2(src + 10 * P + c);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            f[v][3] = v ? q3.y : q3.x;
            f[v][4] = v ? q4.y : q4.x;
            f[v][9] = v ? q9.y : q9.x;
            f[v][10] = v ? q10.y : q10.x;
        }
        f[0][2] = p2.y; f[0][7] = p7.y;
        f[1][2] = r2; f[1][7] = r7;
        if (ic == L.nx - 1) { f[0][2] = 0.0; f[0][7] = 0.0; }
        if (ic + 1 == L.nx - 1) { f[1][2] = 0.0; f[1][7] = 0.0; }
    } else {
        const unsigned short mm = *reinterpret_cast<const unsigned short *>(L.mask + node(L, ic, jc));
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int mat = (mm >> (8 * v)) & 3;
            conductor[v] = mat == MAT_PEC;
            inv_eps[v] = mat_inv_eps(L, mat);
            eps_rest[v] = mat_eps_rest(L, mat);
        }
        // -x populations come from the node on the right; the last node keeps its own
        f[0][2] = p2.y; f[0][7] = p7.y;
        f[1][2] = r2; f[1][7] = r7;
        if (ic == L.nx - 1) { f[0][2] = keep * p2.x; f[0][7] = keep * p7.x; }
        if (ic + 1 == L.nx - 1) { f[1][2] = keep * p2.y; f[1][7] = keep * p7.y; }
        const size_t strip = at(ic, L.ny, L.sf);
        // +y populations come from (i, j - 1)
        if (jc == 0) {
            const Double2 a3 = ld2(src + 3 * P + c), a9 = ld2(src + 9 * P + c);
            const Double2 s3 = ld2(src + 3 * P + strip), s9 = ld2(src + 9 * P + strip);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                f[v][3] = keep * (v ? a3.y : a3.x) + OPEN_DELTA * (v ? s3.y : s3.x);
                f[v][9] = keep * (v ? a9.y : a9.x) + OPEN_DELTA * (v ? s9.y : s9.x);
            }
        } else {
            const Double2 b3 = ld2(src + 3 * P + c - L.sf), b9 = ld2(src + 9 * P + c - L.sf);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                f[v][3] = v ? b3.y : b3.x;
                f[v][9] = v ? b9.y : b9.x;
            }
        }
        // -y populations come from (i, j + 1)
        if (jc == L.ny - 1) {
            const Double2 a4 = ld2(src + 4 * P + c), a10 = ld2(src + 10 * P + c);
            const Double2 s4 = ld2(src + 4 * P + strip), s10 = ld2(src + 10 * P + strip);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                f[v][4] = keep * (v ? a4.y : a4.x) + OPEN_DELTA * (v ? s4.y : s4.x);
                f[v][10] = keep * (v ? a10.y : a10.x) + OPEN_DELTA * (v ? s10.y : s10.x);
            }
        } else {
            const Double2 t4 = ld2(src + 4 * P + c + L.sf), t10 = ld2(src + 10 * P + c + L.sf);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                f[v][4] = v ? t4.y : t4.x;
                f[v][10] = v ? t10.y : t10.x;
            }
        }
    }
    double out[2][11], ez[2], hx[2], hy[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) f64_collide(L, f[v], inv_eps[v], eps_rest[v], conductor[v], out[v], ez[v], hx[v], hy[v]);
    if (!valid) return;
    if (second) {
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            Double2 w;
            w.x = out[0][k];
            w.y = out[1][k];
            put(reinterpret_cast<Double2 *>(dst + k * P + c), w, L.stream_stores);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 11; ++k) put(&dst[k * P + c], out[0][k], L.stream_stores);
    }
    if (fields) {
        const size_t cf = at(ic, jc, L.sfld);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            if (v == 1 && !second) break;
            fields[0 * P + cf + v] = ez[v];
            fields[1 * P + cf + v] = hx[v];
            fields[2 * P + cf + v] = hy[v];
        }
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch.  A launch reads the state at n once and writes the
// state at n + 2 once: the bytes of one step for two lattice updates.
//
// One wavefront is one work item: a strip of 64 columns (one node per lane;
// HX halo columns at each side, 64 - 2 HX output columns) and H output rows.
// Step n -> n + 1 runs on rows j0 - 1 .. j0 + H and every column of the
// strip, step n + 1 -> n + 2 on rows j0 .. j0 + H - 1 and the output
// columns.  The wavefront sweeps the rows holding, at level n, all 11
// populations of the row being updated and of the next one (one or two more
// in flight) and, of the row behind, only the two populations it sends to the
// row being updated; likewise at level n + 1.  x-neighbours come from the
// adjacent lanes through DPP wave shifts.  Rows beyond the domain's edges
// are loaded from a clamped address and never used: edge rows take their
// edge rules instead.  Consecutive row segments sweep in opposite
// directions, so the two segments next to a seam read its rows at the same
// moment.  The companion row is stepped alongside where rows 0 or ny - 1
// need it; the bottom segment's wavefronts store it.
// ---------------------------------------------------------------------------

constexpr int F64_TWO_WAVES = 4;  // independent wavefronts per block

// Lane k receives lane k - 1's (from_left) or lane k + 1's (from_right)
// value; the end lanes receive 0 and are halo columns.
__device__ __forceinline__ double dpp_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double dpp_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The 11 populations of a node at one level.
struct Pops {
    double f[11];
};
// The two populations a row sends to a neighbour row: (f3, f9) up, (f4, f10) down.
struct Send {
    double e, h;
};
__device__ __forceinline__ Send send_up(const Pops &p) { return Send{p.f[3], p.f[9]}; }
__device__ __forceinline__ Send send_down(const Pops &p) { return Send{p.f[4], p.f[10]}; }
// What the companion row sends rows 0 (up) and ny - 1 (down) at one level.
struct StripSend {
    Send up, down;
};

// Gather of node (i, j) from registers: its own populations o and its
// neighbours' streaming ones (left: f1, f6; right: f2, f7; below: f3, f9;
// above: f4, f10), with f64_node's edge rules and operations.  STRIP: the
// companion row (uniform in y, nothing enters on the right).
template <bool STRIP>
__device__ __forceinline__ void f64_gather(const Lattice &L, int i, int j, const Pops &o, double l1, double l6,
                                           double r2, double r7, const Send &below, const Send &above,
                                           const StripSend &strip, double einc, double (&f)[11])
{
#pragma clang fp contract(off)
    const double keep = 1.0 - OPEN_DELTA;
    f[0] = o.f[0];
    f[5] = o.f[5];
    f[8] = o.f[8];
    if (i == 0) { f[1] = einc / 3.0; f[6] = 0.0; }
    else { f[1] = l1; f[6] = l6; }
    if (STRIP) {
        f[3] = o.f[3];
        f[4] = o.f[4];
        f[9] = o.f[9];
        f[10] = o.f[10];
        if (i == L.nx - 1) { f[2] = 0.0; f[7] = 0.0; }
        else { f[2] = r2; f[7] = r7; }
        return;
    }
    if (i == L.nx - 1) { f[2] = keep * o.f[2]; f[7] = keep * o.f[7]; }
    else { f[2] = r2; f[7] = r7; }
    if (j == 0) {
        f[3] = keep * o.f[3] + OPEN_DELTA * strip.up.e;
        f[9] = keep * o.f[9] + OPEN_DELTA * strip.up.h;
    } else { f[3] = below.e; f[9] = below.h; }
    if (j == L.ny - 1) {
        f[4] = keep * o.f[4] + OPEN_DELTA * strip.down.e;
        f[10] = keep * o.f[10] + OPEN_DELTA * strip.down.h;
    } else { f[4] = above.e; f[10] = above.h; }
}

// One row's update at one level (one node per lane): gather, collide; the
// node's fields into fld.
template <bool STRIP>
__device__ __forceinline__ void f64_row_update(const Lattice &L, int i, int j, uint8_t m, const Pops &o,
                                               const Send &below, const Send &above, const StripSend &strip,
                                               double einc, Pops &out, double (&fld)[3])
{
    // x-neighbours across lanes (every lane takes part)
    const double l1 = dpp_from_left(o.f[1]), l6 = dpp_from_left(o.f[6]);
    const double r2 = dpp_from_right(o.f[2]), r7 = dpp_from_right(o.f[7]);
    double inv_eps = 1.0, eps_rest = 1.0 - 2.0 / 3.0;
    bool conductor = false;
    if (!STRIP) {
        const int mat = m & 3;
        conductor = mat == MAT_PEC;
        inv_eps = mat_inv_eps(L, mat);
        eps_rest = mat_eps_rest(L, mat);
    }
    double f[11];
    f64_gather<STRIP>(L, i, j, o, l1, l6, r2, r7, below, above, strip, einc, f);
    f64_collide(L, f, inv_eps, eps_rest, conductor, out.f, fld[0], fld[1], fld[2]);
}

// LA: the load of a row ahead is issued before this row's arithmetic, two
// rows ahead (2) or one (1), hiding its latency inside the wavefront, or
// after it (0, keeping its registers free during the arithmetic so that
// three wavefronts fit a SIMD).
// FL: the field planes of both levels are written (fl1: n + 1, fl2: n + 2),
// every node the launch owns, the companion row included.  one: a single
// step (a solve's last one), whose level n + 1 is the new state.
template <int H, int HX, int LA, bool FL>
__device__ __forceinline__ void f64_two_step_wave(const Lattice &L, const double *__restrict__ src,
                                                  double *__restrict__ dst, double *__restrict__ fl1,
                                                  double *__restrict__ fl2, double einc0, double einc1, int sx,
                                                  int sy, bool one)
{
    constexpr int OW = 64 - 2 * HX;
    static_assert(HX >= 2 && OW > 0, "two-step strip shape");
    const int x0 = sx * OW, j0 = sy * H;
    const int lane = threadIdx.x;
    const int i = x0 - HX + lane;
    const bool out_lane = i >= 0 && i < L.nx && lane >= HX && lane < HX + OW;
    const size_t P = L.plane;
    const int ic = min(max(i, 0), L.nx - 1);
    auto load = [&](int r, Pops &d, uint8_t &m) {
        const int rc = min(max(r, 0), L.ny - 1);
        const double *row = src + (size_t)rc * L.sf + ic;
#pragma unroll
        for (int k = 0; k < 11; ++k) d.f[k] = row[k * P];
        m = L.mask[(size_t)rc * L.pitch + ic];
    };
    auto store = [&](int r, const Pops &d) {
        double *row = dst + (size_t)r * L.sf + i;
#pragma unroll
        for (int k = 0; k < 11; ++k) put(&row[k * P], d.f[k], L.stream_stores);
    };
    auto store_fields = [&](double *fl, int r, const double (&v)[3]) {
        double *p = fl + (size_t)r * L.sfld + i;
        p[0] = v[0];
        p[P] = v[1];
        p[2 * P] = v[2];
    };
    double fld[3];

    // companion row at n and n + 1 where rows 0 or ny - 1 are updated here
    StripSend s0{}, s1{};
    if (j0 <= 1 || j0 + H >= L.ny - 1) {
        Pops c0, c1;
        const double *row = src + (size_t)L.ny * L.sf + ic;
#pragma unroll
        for (int k = 0; k < 11; ++k) c0.f[k] = row[k * P];
        f64_row_update<true>(L, i, L.ny, 0, c0, Send{}, Send{}, StripSend{}, einc0, c1, fld);
        s0 = StripSend{send_up(c0), send_down(c0)};
        s1 = StripSend{send_up(c1), send_down(c1)};
        if (one && j0 == 0 && out_lane) {
            store(L.ny, c1);
            if (FL) store_fields(fl1, L.ny, fld);
        }
        if (!one && j0 == 0) {
            if (FL && out_lane) store_fields(fl1, L.ny, fld);
            Pops c2;
            f64_row_update<true>(L, i, L.ny, 0, c1, Send{}, Send{}, StripSend{}, einc1, c2, fld);
            if (out_lane) store(L.ny, c2);
            if (FL && out_lane) store_fields(fl2, L.ny, fld);
        }
    }

    auto sweep = [&](auto dir_tag) {
        constexpr int DIR = decltype(dir_tag)::value;
        const int first = DIR > 0 ? j0 - 1 : j0 + H;  // first row of step n -> n + 1
        // what a row sends to the row ahead of it / behind it in the sweep
        auto to_ahead = [](const Pops &p) { return DIR > 0 ? send_up(p) : send_down(p); };
        auto to_behind = [](const Pops &p) { return DIR > 0 ? send_down(p) : send_up(p); };
        Pops a_cur, a_ahead, a_far, tmp;
        uint8_t m_cur, m_ahead, m_far = 0, m_prev = 0, m_dummy;
        load(first - DIR, tmp, m_dummy);
        Send a_behind = to_ahead(tmp);
        load(first, a_cur, m_cur);
        load(first + DIR, a_ahead, m_ahead);
        if constexpr (LA == 2) load(first + 2 * DIR, a_far, m_far);
        Send b_behind{};
        Pops b_cur{};
        // unrolled whole: the rows in flight then rotate through registers
        // instead of being copied, which would wait for their loads
#pragma unroll
        for (int k = 0; k < H + 2; ++k) {
            const int r1 = first + DIR * k;
            Pops a_next;
            uint8_t m_next = 0;
            if constexpr (LA == 2) {
                // rows up to first + (H + 2) DIR are read, as with LA = 1
                a_next = a_far;
                m_next = m_far;
                if (k < H) load(r1 + 3 * DIR, a_far, m_far);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (LA == 1) {
                if (k <= H) load(r1 + 2 * DIR, a_next, m_next);
                else { a_next = a_ahead; m_next = m_ahead; }
                // keep the look-ahead load ahead of this row's arithmetic
                __builtin_amdgcn_sched_barrier(0);
            }
            // step n -> n + 1 on row r1
            Pops b_new;
            const Send a_side = to_behind(a_ahead);
            f64_row_update<false>(L, i, r1, m_cur, a_cur, DIR > 0 ? a_behind : a_side, DIR > 0 ? a_side : a_behind,
                                  s0, einc0, b_new, fld);
            if (out_lane && r1 >= j0 && r1 < j0 + H && r1 < L.ny) {
                if (FL) store_fields(fl1, r1, fld);
                if (one) store(r1, b_new);  // a single step: this row's result is the new state
            }
            // step n + 1 -> n + 2 on the row behind r1
            if (!one && k >= 2) {
                const int r2 = r1 - DIR;
                Pops o;
                const Send b_side = to_behind(b_new);
                f64_row_update<false>(L, i, r2, m_prev, b_cur, DIR > 0 ? b_behind : b_side,
                                      DIR > 0 ? b_side : b_behind, s1, einc1, o, fld);
                if (out_lane && r2 < L.ny) {
                    store(r2, o);
                    if (FL) store_fields(fl2, r2, fld);
                }
            }
            if constexpr (LA == 0) {
                if (k <= H) load(r1 + 2 * DIR, a_next, m_next);
                else { a_next = a_ahead; m_next = m_ahead; }
            }
            b_behind = to_ahead(b_cur);
            b_cur = b_new;
            m_prev = m_cur;
            a_behind = to_ahead(a_cur);
            a_cur = a_ahead;
            m_cur = m_ahead;
            a_ahead = a_next;
            m_ahead = m_next;
        }
    };
    if (sy & 1) sweep(std::integral_constant<int, -1>{});
    else sweep(std::integral_constant<int, 1>{});
}

// W: wavefronts per SIMD the register allocation must allow (2: up to 256
// VGPRs; 3: up to 168).
template <int H, int HX, int W, int LA, bool FL>
__global__ __launch_bounds__(64 * F64_TWO_WAVES, W) void k_step2_f64(Lattice L, const double *__restrict__ src,
                                                                     double *__restrict__ dst, double *__restrict__ fl1,
                                                                     double *__restrict__ fl2, double einc0,
                                                                     double einc1, int nsx, int nsy)
{
    // Work order as for the FP32 / BF16 two-step kernels: a cache-resident
    // state takes the segments of one strip in turn, XCD-contiguous; a state
    // streamed from HBM takes whole bands of rows.
    const int nb = gridDim.x;
    const int b = L.stream_stores ? (int)blockIdx.x : xcd_tile(blockIdx.x, nb);
    const int w = __builtin_amdgcn_readfirstlane(b * F64_TWO_WAVES + (int)threadIdx.y);
    if (w >= nsx * nsy) return;  // whole wavefront
    const int sx = L.stream_stores ? w % nsx : w / nsy, sy = L.stream_stores ? w / nsx : w % nsy;
    f64_two_step_wave<H, HX, LA, FL>(L, src, dst, fl1, fl2, einc0, einc1, sx, sy, false);
}

// Batched two-step launch: wavefront w takes items[w] (slot, strip, row
// segment) of a resident FP64 solve at that solve's own step n; the field
// planes of both levels (by level parity) when either is averaged; a single
// step when the solve has one left.
template <int H, int HX, int W, int LA>
__global__ __launch_bounds__(64 * F64_TWO_WAVES, W) void k_step2_f64_batch(SolveDesc *__restrict__ D,
                                                                           const Tile *__restrict__ items, int nitems,
                                                                           int remap)
{
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(b * F64_TWO_WAVES + (int)threadIdx.y);
    if (w >= nitems) return;
    const Tile t = items[w];
    const SolveDesc &d = D[t.slot];
    const int64_t n = d.n;
    if (n >= d.steps) return;
    const bool one = d.steps - n == 1;
    const double e0 = batch_incident(d, n), e1 = one ? 0.0 : batch_incident(d, n + 1);
    const double *src = (const double *)d.state[d.cur];
    double *dst = (double *)d.state[d.cur ^ 1];
    if (n + 2 > d.steps - d.window) {
        double *fl1 = d.fields + (size_t)((n + 1) & 1) * d.fields_level;
        double *fl2 = d.fields + (size_t)((n + 2) & 1) * d.fields_level;
        f64_two_step_wave<H, HX, LA, true>(d.L, src, dst, fl1, fl2, e0, e1, t.tx, t.ty, one);
    } else {
        f64_two_step_wave<H, HX, LA, false>(d.L, src, dst, nullptr, nullptr, e0, e1, t.tx, t.ty, one);
    }
}

template <typename F> void f64_two_dispatch(int variant, F &&go)
{
    using H6 = std::integral_constant<int, 6>;
    using H8 = std::integral_constant<int, 8>;
    using H10 = std::integral_constant<int, 10>;
    using H12 = std::integral_constant<int, 12>;
    using X4 = std::integral_constant<int, 4>;
    using X8 = std::integral_constant<int, 8>;
    using W2 = std::integral_constant<int, 2>;
    using W3 = std::integral_constant<int, 3>;
    using A0 = std::integral_constant<int, 0>;
    using A1 = std::integral_constant<int, 1>;
    using A2 = std::integral_constant<int, 2>;
    switch (variant) {
    case F64_TWO_H10_X4: go(H10{}, X4{}, W2{}, A1{}); break;
    case F64_TWO_H12_X4: go(H12{}, X4{}, W2{}, A1{}); break;
    case F64_TWO_H12_X4_W3: go(H12{}, X4{}, W3{}, A0{}); break;
    case F64_TWO_H12_X4_LA2: go(H12{}, X4{}, W2{}, A2{}); break;
    case F64_TWO_H6_X8: go(H6{}, X8{}, W2{}, A1{}); break;
    case F64_TWO_H8_X8: go(H8{}, X8{}, W2{}, A1{}); break;
    case F64_TWO_H8_X8_LA2: go(H8{}, X8{}, W2{}, A2{}); break;
    default: go(H12{}, X8{}, W2{}, A1{}); break;
    }
}

}  // namespace

void two_step_shape_f64(int variant, int nx, int ny, int &nsx, int &nsy)
{
    f64_two_dispatch(variant, [&](auto htag, auto xtag, auto, auto) {
        constexpr int H = decltype(htag)::value, HX = decltype(xtag)::value;
        nsx = (nx + (64 - 2 * HX) - 1) / (64 - 2 * HX);
        nsy = (ny + H - 1) / H;
    });
}

hipError_t launch_step2_f64_batch(int variant, SolveDesc *d, const Tile *items, int nitems, int remap, hipStream_t s)
{
    if (variant < 0 || variant >= F64_TWO_STEP_VARIANTS) return hipErrorInvalidValue;
    if (nitems <= 0) return hipSuccess;
    const int blocks = (nitems + F64_TWO_WAVES - 1) / F64_TWO_WAVES;
    f64_two_dispatch(variant, [&](auto htag, auto xtag, auto wtag, auto atag) {
        constexpr int H = decltype(htag)::value, HX = decltype(xtag)::value, W = decltype(wtag)::value;
        constexpr int LA = decltype(atag)::value;
        hipLaunchKernelGGL((k_step2_f64_batch<H, HX, W, LA>), dim3(blocks), dim3(64, F64_TWO_WAVES), 0, s, d, items,
                           nitems, remap);
    });
    return hipGetLastError();
}

hipError_t launch_step_f64(const Lattice &L, const double *src, double *dst, double *fields, double einc,
                           hipStream_t s, int variant)
{
    auto grid = [&](int cx, int r) { return dim3((L.nx + cx - 1) / cx, (L.ny + 1 + r - 1) / r); };
    // two nodes per thread: each block covers twice its width in columns
    auto grid2 = [&](int cx, int r) { return dim3((L.nx + 2 * cx - 1) / (2 * cx), (L.ny + 1 + r - 1) / r); };
    switch (variant) {
    case F64_W256_R1: hipLaunchKernelGGL((k_step_f64<256, 1>), grid(256, 1), dim3(256, 1), 0, s, L, src, dst, fields, einc); break;
    case F64_W256_R2: hipLaunchKernelGGL((k_step_f64<256, 2>), grid(256, 2), dim3(256, 2), 0, s, L, src, dst, fields, einc); break;
    case F64_PAIR_R4: hipLaunchKernelGGL((k_step_f64_pair<BX, 4>), grid2(BX, 4), dim3(BX, 4), 0, s, L, src, dst, fields, einc); break;
    case F64_PAIR_W256_R1: hipLaunchKernelGGL((k_step_f64_pair<256, 1>), grid2(256, 1), dim3(256, 1), 0, s, L, src, dst, fields, einc); break;
    default: hipLaunchKernelGGL((k_step_f64<BX, 4>), grid(BX, 4), dim3(BX, 4), 0, s, L, src, dst, fields, einc); break;
    }
    return hipGetLastError();
}

hipError_t launch_step2_f64(const Lattice &L, const double *src, double *dst, double einc0, double einc1,
                            double *fields1, double *fields2, hipStream_t s, int variant)
{
    if (variant < 0 || variant >= F64_TWO_STEP_VARIANTS || src == dst) return hipErrorInvalidValue;
    if ((fields1 == nullptr) != (fields2 == nullptr) || (fields1 && fields1 == fields2)) return hipErrorInvalidValue;
    f64_two_dispatch(variant, [&](auto htag, auto xtag, auto wtag, auto atag) {
        constexpr int H = decltype(htag)::value, HX = decltype(xtag)::value, W = decltype(wtag)::value;
        constexpr int LA = decltype(atag)::value;
        const int nsx = (L.nx + (64 - 2 * HX) - 1) / (64 - 2 * HX);
        const int nsy = (L.ny + H - 1) / H;
        const int blocks = (nsx * nsy + F64_TWO_WAVES - 1) / F64_TWO_WAVES;
        if (fields1)
            hipLaunchKernelGGL((k_step2_f64<H, HX, W, LA, true>), dim3(blocks), dim3(64, F64_TWO_WAVES), 0, s, L, src, dst,
                               fields1, fields2, einc0, einc1, nsx, nsy);
        else
            hipLaunchKernelGGL((k_step2_f64<H, HX, W, LA, false>), dim3(blocks), dim3(64, F64_TWO_WAVES), 0, s, L, src,
                               dst, nullptr, nullptr, einc0, einc1, nsx, nsy);
    });
    return hipGetLastError();
}

}  // namespace jlb
