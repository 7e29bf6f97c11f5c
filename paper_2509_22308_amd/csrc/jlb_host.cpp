// Host side of the Janus-cylinder EM lattice Boltzmann library: problem
// checks, staircase geometry, contour table, workspace layout and the
// time-stepping driver behind the C ABI of include/jlb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/jlb.h"
#include "jlb_host_internal.h"
#include "jlb_internal.h"

namespace jlb {

static_assert(JLB_STEP_VARIANTS == NEQ_VARIANTS, "single-step variant count");
static_assert(JLB_FP64_STEP_VARIANTS == F64_VARIANTS, "FP64 variant count");
static_assert(JLB_TWO_STEP_VARIANTS == TWO_STEP_VARIANTS, "two-step variant count");
static_assert(JLB_FP64_TWO_STEP_VARIANTS == F64_TWO_STEP_VARIANTS, "FP64 two-step variant count");
static_assert(JLB_STATIC_SCRATCH_BYTES == STATIC_SCRATCH_BYTES, "library-held scratch size");

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }
const char *last_error() { return g_last_error.c_str(); }

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(JLB_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// Problem plan: every derived quantity of one solve
// ---------------------------------------------------------------------------

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int make_plan(const jlb_problem *p, Plan *pl)
{
    if (!p || !pl) return fail(JLB_E_ARG, "null problem or plan");
    if (p->nx < 16 || p->ny < 16) return fail(JLB_E_ARG, "grid %dx%d smaller than 16x16", p->nx, p->ny);
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(JLB_E_ARG, "grid too large");
    if (p->kind < 0 || p->kind > 2) return fail(JLB_E_ARG, "unknown kind %d", p->kind);
    if (p->precision < 0 || p->precision > 2) return fail(JLB_E_ARG, "unknown precision %d", p->precision);
    if (!(p->radius > 0.0)) return fail(JLB_E_ARG, "radius must be > 0");
    if (!(p->plateau_tol >= 0.0) || !std::isfinite(p->plateau_tol)) return fail(JLB_E_ARG, "plateau_tol must be >= 0");
    if (!(p->eps1 >= 1.0) || !std::isfinite(p->eps1)) return fail(JLB_E_ARG, "eps1 must be >= 1");
    if (p->kind == JLB_DIELECTRIC_JANUS && (!(p->eps2 >= 1.0) || !std::isfinite(p->eps2)))
        return fail(JLB_E_ARG, "eps2 must be >= 1");
    if (!std::isfinite(p->phi0)) return fail(JLB_E_ARG, "phi0 not finite");
    if (!(p->wavelength > 0.0) || !std::isfinite(p->wavelength)) return fail(JLB_E_ARG, "wavelength must be > 0");
    const double period = 3.0 * p->wavelength;
    const int64_t T = (int64_t)std::llround(period);
    if (std::fabs(period - (double)T) > 1e-9 || T < 4) return fail(JLB_E_ARG, "3*wavelength must be an integer >= 4");
    if (!(p->e0 > 0.0) || !std::isfinite(p->e0)) return fail(JLB_E_ARG, "e0 must be > 0");
    if (p->steps < 1) return fail(JLB_E_ARG, "steps must be >= 1");
    if (p->avg_periods < 1 || p->ramp_periods < 0) return fail(JLB_E_ARG, "avg_periods >= 1 and ramp_periods >= 0");
    if (!(p->contour_offset > 1.5)) return fail(JLB_E_GEOMETRY, "contour_offset must exceed 1.5 cells");
    if (p->contour_points < 0) return fail(JLB_E_ARG, "contour_points must be >= 0");
    if (p->polarization != JLB_TM && p->polarization != JLB_TE) return fail(JLB_E_ARG, "polarization must be 0 (TM) or 1 (TE)");

    Plan &q = *pl;
    q.prob = *p;
    q.nx = p->nx;
    q.ny = p->ny;
    q.pitch = (int)align_up((size_t)p->nx, ROW_ALIGN);
    q.plane = (size_t)(p->ny + 1) * q.pitch;
    q.period = period;
    q.T = T;
    q.omega = 2.0 * M_PI / period;
    q.ramp_steps = (double)p->ramp_periods * period;
    q.window = (int64_t)p->avg_periods * T;
    q.cx = 0.5 * (p->nx - 1);
    q.cy = 0.5 * (p->ny - 1);
    if (p->flags & JLB_F_CENTRE) {
        if (!std::isfinite(p->cx) || !std::isfinite(p->cy)) return fail(JLB_E_ARG, "centre (cx, cy) not finite");
        q.cx = p->cx;
        q.cy = p->cy;
    }
    q.rc = p->radius + p->contour_offset;
    q.nc = p->contour_points > 0 ? p->contour_points : 8 * (int)std::ceil(2.0 * M_PI * q.rc / 8.0);
    // disk, contour and a 4-cell margin inside the grid
    const double reach = q.rc + 4.0;
    if (q.cx - reach < 0.0 || q.cy - reach < 0.0 || q.cx + reach > p->nx - 1 || q.cy + reach > p->ny - 1)
        return fail(JLB_E_GEOMETRY, "disk radius %.3g + contour offset %.3g + 4 around (%.3g, %.3g) does not fit a %dx%d grid",
                    p->radius, p->contour_offset, q.cx, q.cy, p->nx, p->ny);
    double eps_max = p->eps1;
    if (p->kind == JLB_DIELECTRIC_JANUS) eps_max = std::max(eps_max, p->eps2);
    if (!(p->flags & JLB_F_ALLOW_UNDERRESOLVED) && p->wavelength / std::sqrt(eps_max) < 10.0)
        return fail(JLB_E_RESOLUTION, "lambda/sqrt(eps_max) = %.3g < 10", p->wavelength / std::sqrt(eps_max));
    if (p->steps < (int64_t)(p->avg_periods + p->ramp_periods) * T)
        return fail(JLB_E_WINDOW, "steps %lld < (avg_periods + ramp_periods) * T = %lld", (long long)p->steps,
                    (long long)(p->avg_periods + p->ramp_periods) * T);

    q.eps[MAT_VACUUM] = 1.0;
    q.eps[MAT_REGION2] = p->eps1;
    q.eps[MAT_REGION3] = p->kind == JLB_DIELECTRIC_JANUS ? p->eps2 : (p->kind == JLB_HOMOGENEOUS ? p->eps1 : 1.0);
    q.eps[MAT_PEC] = 1.0;

    // workspace layout (each region 256-byte aligned)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    if (p->precision == JLB_FP64) {
        q.state_bytes = 11 * q.plane * sizeof(double);
        q.bytes_per_lup = 11 * 2 * sizeof(double) + 1;
    } else {
        const size_t nb = p->precision == JLB_FP32 ? 4 : 2;
        q.state_bytes = 3 * q.plane * sizeof(float) + 8 * q.plane * nb;
        q.bytes_per_lup = (3 * 4 + 8 * nb) * 2 + 1;
    }
    q.off_state[0] = take(q.state_bytes);
    q.off_state[1] = take(q.state_bytes);
    // FP64: field planes for two time levels, by parity (a launch that writes
    // level n + 1 leaves level n intact)
    q.off_fields = p->precision == JLB_FP64 ? take(2 * 3 * q.plane * sizeof(double)) : 0;
    // FP32 / BF16: fields at the middle level of a two-step launch, written
    // only at the contour-stencil nodes
    // contour-stencil fields of up to three intermediate levels (a four-step
    // launch inside the window; a two-step launch uses the first)
    q.off_mid = p->precision == JLB_FP64 ? 0 : take((size_t)3 * 3 * q.pitch * q.ny * sizeof(float));
    q.off_mask = take((size_t)q.ny * q.pitch);
    q.off_i0 = take(q.nc * sizeof(int));
    q.off_j0 = take(q.nc * sizeof(int));
    q.off_wx = take(q.nc * sizeof(double));
    q.off_wy = take(q.nc * sizeof(double));
    q.off_nxk = take(q.nc * sizeof(double));
    q.off_nyk = take(q.nc * sizeof(double));
    q.off_acc = take(4 * q.nc * sizeof(double));
    q.off_dft = take(12 * q.nc * sizeof(double));  // far-field phasor sums
    q.off_out = take(8 * sizeof(double));
    Lattice tmp{};
    tmp.nx = q.nx;
    tmp.ny = q.ny;
    q.nparts = energy_partials(tmp);
    q.off_parts = take(q.nparts * sizeof(double));
    q.ws_bytes = off;
    return JLB_OK;
}

// ---------------------------------------------------------------------------
// Geometry (Sec. II, Fig. schematic): staircase material map on the nodes
// ---------------------------------------------------------------------------

void material_map(const Plan &q, uint8_t *mat, size_t row_stride)
{
    const jlb_problem &p = q.prob;
    const double sp = std::sin(p.phi0), cp = std::cos(p.phi0);
    for (int j = 0; j < q.ny; ++j) {
        for (int i = 0; i < q.nx; ++i) {
            const double dx = i - q.cx, dy = j - q.cy;
            uint8_t m = MAT_VACUUM;
            if (dx * dx + dy * dy <= p.radius * p.radius) {
                if (p.kind == JLB_HOMOGENEOUS) {
                    m = MAT_REGION2;
                } else {
                    // side of the interface diameter: region II towards (-sin phi0, -cos phi0)
                    const double s = -dx * sp - dy * cp;
                    m = s > 1e-9 ? MAT_REGION2 : (p.kind == JLB_DIELECTRIC_JANUS ? MAT_REGION3 : MAT_PEC);
                }
            }
            mat[(size_t)j * row_stride + i] = m;
        }
    }
}

// Mask bytes: the material id (the contour-stencil bit is added with the
// contour table).
void build_mask(const Plan &q, std::vector<uint8_t> &mask)
{
    mask.assign((size_t)q.ny * q.pitch, 0);
    material_map(q, mask.data(), q.pitch);
}

// Contour (Sec. II.B): N_c midpoint samples on the circle of radius R_c.
void build_contour(const Plan &q, ContourHost &c)
{
    c.i0.resize(q.nc);
    c.j0.resize(q.nc);
    c.wx.resize(q.nc);
    c.wy.resize(q.nc);
    c.nxk.resize(q.nc);
    c.nyk.resize(q.nc);
    for (int k = 0; k < q.nc; ++k) {
        const double th = 2.0 * M_PI * (k + 0.5) / q.nc;
        c.nxk[k] = std::cos(th);
        c.nyk[k] = std::sin(th);
        const double px = q.cx + q.rc * c.nxk[k];
        const double py = q.cy + q.rc * c.nyk[k];
        c.i0[k] = (int)std::floor(px);
        c.j0[k] = (int)std::floor(py);
        c.wx[k] = px - c.i0[k];
        c.wy[k] = py - c.j0[k];
    }
}

// Incident wave at the left edge (Sec. III): E_inc(n) = E0 r(n) cos(omega n),
// raised-cosine ramp r over the first ramp_periods periods.  The phase is
// taken as omega (n mod T), which repeats exactly with the period, so the
// source values captured in a graph of whole periods equal those of direct
// launches at every replay.
double incident(const Plan &q, int64_t n)
{
    double ramp = 1.0;
    if (q.prob.ramp_periods > 0 && (double)n < q.ramp_steps) ramp = 0.5 * (1.0 - std::cos(M_PI * (double)n / q.ramp_steps));
    return q.prob.e0 * ramp * std::cos(q.omega * (double)(n % q.T));
}

// ---------------------------------------------------------------------------
// Step-kernel variant per precision (FP32, BF16); set by the autotuner or
// forced by the caller.  All variants give identical results.
// ---------------------------------------------------------------------------

static std::atomic<int> g_variant[3] = {{0}, {NEQ_DIRECT}, {NEQ_DIRECT}};
// Two-step kernel variant per precision, -1 = off (FP64: F64TwoStepVariant,
// used for the graph-replayed periods before the averaging window).
static std::atomic<int> g_two[3] = {{F64_TWO_H10_X4}, {TWO_V1_H8_X8}, {TWO_V1_H8_X8}};

int step_variant(int precision) { return g_variant[precision].load(std::memory_order_relaxed); }
void set_step_variant(int precision, int v) { g_variant[precision].store(v, std::memory_order_relaxed); }
int two_step_variant(int precision) { return g_two[precision].load(std::memory_order_relaxed); }
static void set_two_step_variant(int precision, int v) { g_two[precision].store(v, std::memory_order_relaxed); }
// Multi-step (three or four steps per launch) kernel variant per precision
// for the graph-captured periods and the ramp of a single solve, -1 = off.
static std::atomic<int> g_multi[3] = {{-1}, {MULTI_S4_H10_X4}, {MULTI_S4_H10_X4}};
int multi_step_variant(int precision) { return g_multi[precision].load(std::memory_order_relaxed); }
static void set_multi_step_variant(int precision, int v) { g_multi[precision].store(v, std::memory_order_relaxed); }

hipError_t launch_step(const Plan &q, const Lattice &L, void *src, void *dst, double *fields, double einc, hipStream_t s,
                       int variant)
{
    if (q.prob.precision == JLB_FP64) return launch_step_f64(L, (const double *)src, (double *)dst, fields, einc, s, variant);
    return launch_step_neq(q.prob.precision, L, src, dst, einc, s, variant);
}

// ---------------------------------------------------------------------------
// Streams
// ---------------------------------------------------------------------------

hipStream_t own_stream()
{
    static thread_local hipStream_t s = nullptr;
    static thread_local int dev = -1;
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return nullptr;
    if (!s || dev != d) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        dev = d;
    }
    return s;
}

// ---------------------------------------------------------------------------
// One solve on prepared device memory
// ---------------------------------------------------------------------------

// Largest state pair (both buffers) a single solve runs cache-resident:
// ordinary stores and the XCD-contiguous work order; larger ones stream
// their stores past the caches in plain order.  FP32 / BF16 sweeps stay
// faster resident up to 192 MiB (7-15 % at 174-190 MiB, measured against
// streaming); the FP64 two-step sweep already ran 2.5 % slower resident at
// 185 MiB (1024^2), so FP64 switches at 160 MiB.
size_t resident_limit(int precision)
{
    return precision == JLB_FP64 ? CACHE_RESIDENT_BYTES : (size_t)192 << 20;
}

Lattice lattice_of(const Plan &q, const uint8_t *dmask)
{
    Lattice L{};
    L.nx = q.nx;
    L.ny = q.ny;
    L.pitch = q.pitch;
    // row-interleaved planes: plane offset = pitch inside each row
    L.plane = (size_t)q.pitch;
    if (q.prob.precision == JLB_FP64) {
        L.sf = L.sn = 11 * (size_t)q.pitch;
        L.sfld = 3 * (size_t)q.pitch;
    } else {
        const size_t nb = q.prob.precision == JLB_FP32 ? 4 : 2;
        const size_t row_bytes = (3 * 4 + 8 * nb) * (size_t)q.pitch;
        L.sf = row_bytes / 4;
        L.sn = row_bytes / nb;
        L.sfld = L.sf;
    }
    L.mask = dmask;
    for (int k = 0; k < 4; ++k) {
        L.eps[k] = q.eps[k];
        L.eps_rest[k] = q.eps[k] - 2.0 / 3.0;
        L.inv_eps[k] = 1.0 / q.eps[k];
        // FP32 / BF16 states keep one sixth of the fields: the coefficients
        // carry the factor
        L.inv_eps_f[k] = (float)(1.0 / (6.0 * q.eps[k]));
        L.eps_rest_f[k] = (float)(6.0 * L.eps_rest[k]);
    }
    // a conductor node's electric field is zero (Sec. II: E_z^tot = 0), the
    // update's limit of infinite permittivity; the FP64 kernel sets it to 0
    // after the moment, as the oracle does
    L.inv_eps_f[MAT_PEC] = 0.0f;
    L.eps_rest_f[MAT_PEC] = 0.0f;
    L.te = q.prob.polarization == JLB_TE ? 1 : 0;
    L.stream_stores = 2 * q.state_bytes > resident_limit(q.prob.precision) ? 1 : 0;
    return L;
}

ContourDev contour_of(const Plan &q, char *ws)
{
    ContourDev C{};
    C.n = q.nc;
    C.rc = q.rc;
    C.i0 = (const int *)(ws + q.off_i0);
    C.j0 = (const int *)(ws + q.off_j0);
    C.wx = (const double *)(ws + q.off_wx);
    C.wy = (const double *)(ws + q.off_wy);
    C.nxk = (const double *)(ws + q.off_nxk);
    C.nyk = (const double *)(ws + q.off_nyk);
    C.acc = (double *)(ws + q.off_acc);
    return C;
}

void prepare_upload(const Plan &q, std::vector<uint8_t> &img)
{
    // the mask and the contour tables sit back to back in the workspace
    // (off_mask .. off_acc): one host image of that range, one copy
    const size_t lo = q.off_mask, hi = q.off_acc;
    img.assign(hi - lo, 0);
    std::vector<uint8_t> mask;
    build_mask(q, mask);
    ContourHost ch;
    build_contour(q, ch);
    for (int k = 0; k < q.nc; ++k)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) mask[(size_t)(ch.j0[k] + dj) * q.pitch + ch.i0[k] + di] |= MASK_CONTOUR;
    auto put = [&](size_t off, const void *src, size_t bytes) { memcpy(img.data() + (off - lo), src, bytes); };
    put(q.off_mask, mask.data(), mask.size());
    put(q.off_i0, ch.i0.data(), q.nc * sizeof(int));
    put(q.off_j0, ch.j0.data(), q.nc * sizeof(int));
    put(q.off_wx, ch.wx.data(), q.nc * sizeof(double));
    put(q.off_wy, ch.wy.data(), q.nc * sizeof(double));
    put(q.off_nxk, ch.nxk.data(), q.nc * sizeof(double));
    put(q.off_nyk, ch.nyk.data(), q.nc * sizeof(double));
}

int enqueue_upload(const Plan &q, char *ws, hipStream_t s, const std::vector<uint8_t> &img)
{
    HIP_TRY(hipMemcpyAsync(ws + q.off_mask, img.data(), img.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(ws + q.off_state[0], 0, q.state_bytes, s));
    HIP_TRY(hipMemsetAsync(ws + q.off_state[1], 0, q.state_bytes, s));
    if (q.prob.precision == JLB_FP64) HIP_TRY(hipMemsetAsync(ws + q.off_fields, 0, 2 * 3 * q.plane * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(ws + q.off_acc, 0, 4 * q.nc * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(ws + q.off_dft, 0, 12 * q.nc * sizeof(double), s));
    return JLB_OK;
}

int upload_setup(const Plan &q, char *ws, hipStream_t s)
{
    std::vector<uint8_t> img;
    prepare_upload(q, img);
    int rc = enqueue_upload(q, ws, s, img);
    if (rc) return rc;
    // the host image is released on return: finish the copy first
    HIP_TRY(hipStreamSynchronize(s));
    return JLB_OK;
}

// Fields at time level t: FP64 keeps them in the field planes of parity t,
// FP32 / BF16 in the state buffer of parity t.
const void *fields_ptr(const Plan &q, char *ws, int64_t t)
{
    if (q.prob.precision == JLB_FP64) return ws + q.off_fields + (size_t)(t & 1) * 3 * q.plane * sizeof(double);
    return ws + q.off_state[t & 1];
}

// Launches lattice step n (state at n in buffer n % 2 -> state at n + 1) and,
// when `contour` is set, the contour accumulation of time level n + 1.  The
// averaged levels are the last `window` ones, steps - window + 1 .. steps.
static int launch_one_step(const Plan &q, char *ws, const Lattice &L, const ContourDev &C, int64_t n, bool contour,
                           bool want_fields, double einc, hipStream_t s)
{
    const int prec = q.prob.precision;
    void *src = ws + q.off_state[n & 1];
    void *dst = ws + q.off_state[(n + 1) & 1];
    hipError_t e;
    if (prec == JLB_FP64) {
        double *fields = (contour || want_fields) ? (double *)fields_ptr(q, ws, n + 1) : nullptr;
        e = launch_step_f64(L, (const double *)src, (double *)dst, fields, einc, s, step_variant(prec));
    } else {
        e = launch_step_neq(prec, L, src, dst, einc, s, step_variant(prec));
    }
    if (e == hipSuccess && contour) e = launch_contour(prec, L, fields_ptr(q, ws, n + 1), C, s);
    if (e != hipSuccess) return fail(JLB_E_DEVICE, "launch of step %lld failed: %s", (long long)n, hipGetErrorString(e));
    return JLB_OK;
}

int run_solve(const Plan &q, char *ws, jlb_result *res, double *ez, double *hx, double *hy, double *energy,
              hipStream_t s, FarOut far, bool events)
{
    const auto t0 = std::chrono::steady_clock::now();
    memset(res, 0, sizeof(*res));
    int rc = upload_setup(q, ws, s);
    if (rc) return rc;
    const Lattice L = lattice_of(q, (const uint8_t *)(ws + q.off_mask));
    const ContourDev C = contour_of(q, ws);
    int64_t steps = q.prob.steps;
    int64_t wstart = steps - q.window;  // launches from here on produce averaged levels
    const bool use_graph = !(q.prob.flags & JLB_F_NO_GRAPH) && !energy && !far.force;
    // whole periods, a multiple of 4 steps: two-step launches then come in
    // pairs and a chunk leaves state n in buffer n % 2, as single steps do;
    // it is also the spacing of the plateau check points
    const int64_t chunk = q.T % 4 == 0 ? q.T : q.T % 2 == 0 ? 2 * q.T : 4 * q.T;
    // two-step kernels (FP64: not with the plateau search, whose check
    // points read the field planes of single levels)
    const bool f64 = q.prob.precision == JLB_FP64;
    const int two = f64 && q.prob.plateau_tol > 0.0 ? -1 : two_step_variant(q.prob.precision);
    auto two_in = [&](int) { return two >= 0; };
    // multi-step kernels (depth S) for the captured chunks: chunk / S launches
    // must be a whole, even number (the chunk then leaves state n in buffer
    // n % 2), and a row segment must not reach both the bottom and the top row
    int multi = q.prob.precision == JLB_FP64 ? -1 : multi_step_variant(q.prob.precision);
    int depth = 0, mrows = 0;
    if (multi >= 0) multi_step_shape(multi, depth, mrows);
    if (multi >= 0 && depth == 4 && chunk % 8 != 0) {
        // a chunk of 4 (mod 8) steps: three steps per launch (whole-step
        // wavelengths give periods that are multiples of 3, chunks of 12)
        multi = MULTI_S3_H10_X4;
        multi_step_shape(multi, depth, mrows);
    }
    if (multi >= 0 && (chunk % (2 * depth) != 0 || q.ny < mrows + depth)) multi = -1;
    const int64_t ramp_end = (int64_t)std::ceil(q.ramp_steps);
    bool plateau = q.prob.plateau_tol > 0.0;
    double w_prev = -1.0;
    // is level t a plateau check point?
    auto check_level = [&](int64_t t) { return plateau && t >= ramp_end + chunk && (t - ramp_end) % chunk == 0; };
    // energy at level t (whose fields are in place); may end the plateau search
    auto plateau_check = [&](int64_t t) -> int {
        double *slot = (double *)(ws + q.off_out) + 7;
        hipError_t e = launch_energy(q.prob.precision, L, fields_ptr(q, ws, t), (double *)(ws + q.off_parts), q.nparts,
                                     slot, s);
        double w = 0.0;
        if (e == hipSuccess) e = hipMemcpyAsync(&w, slot, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(JLB_E_DEVICE, "plateau check: %s", hipGetErrorString(e));
        if (w_prev >= 0.0 && std::fabs(w - w_prev) <= q.prob.plateau_tol * w && t + q.window <= q.prob.steps) {
            steps = t + q.window;
            wstart = t;
            plateau = false;
        }
        w_prev = w;
        return JLB_OK;
    };

    // timing events (a solve that may not create device objects runs without
    // them: its loop time is then the host's, and the pre-window stretch is
    // not timed)
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evm0 = nullptr, evm1 = nullptr;
    if (events) {
        HIP_TRY(hipEventCreate(&ev0));
        HIP_TRY(hipEventCreate(&ev1));
        HIP_TRY(hipEventCreate(&evm0));
        HIP_TRY(hipEventCreate(&evm1));
        HIP_TRY(hipEventRecord(ev0, s));
    }
    const auto loop_t0 = std::chrono::steady_clock::now();
    // the graph-replayed periods before the window: which kernel, how many launches
    const int main_kind = multi >= 0 ? 3 : two >= 0 ? 2 : 1;
    const int main_variant = multi >= 0 ? multi : two >= 0 ? two : step_variant(q.prob.precision);
    const int64_t main_per_chunk = multi >= 0 ? chunk / depth : two >= 0 ? chunk / 2 : chunk;
    int64_t main_launches = 0;

    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // [0] outside the window, [1] inside
    int64_t gstart[2] = {-1, -1};
    auto capture = [&](int which, int64_t n0) -> int {
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        if (multi >= 0) {
            // launch m takes state n0 + S m from buffer (n0 + m) % 2 to the
            // other one; inside the window it also leaves the contour-stencil
            // fields of levels n0 + S m + 1 .. + S - 1 in mid, and all S levels
            // are accumulated after it
            float *mid = (float *)(ws + q.off_mid);
            const size_t mid_level = (size_t)3 * q.pitch * q.ny;
            for (int64_t m = 0; m < chunk / depth; ++m) {
                const int64_t n = n0 + depth * m;
                double einc[4];
                for (int k = 0; k < depth; ++k) einc[k] = incident(q, n + k);
                void *dst = ws + q.off_state[(n0 + m + 1) & 1];
                hipError_t e = launch_stepm_neq(q.prob.precision, L, ws + q.off_state[(n0 + m) & 1], dst, einc,
                                                which == 1 ? mid : nullptr, mid_level, s, multi);
                if (e == hipSuccess && which == 1) e = launch_contourm(L, mid, mid_level, depth - 1, dst, C, s);
                if (e != hipSuccess) {
                    hipGraph_t dummy;
                    (void)hipStreamEndCapture(s, &dummy);
                    return fail(JLB_E_DEVICE, "multi-step launch: %s", hipGetErrorString(e));
                }
            }
        } else if (two_in(which)) {
            // launch m takes state n0 + 2m from buffer (n0 + m) % 2 to the
            // other one; inside the window it also leaves the fields of level
            // n0 + 2m + 1 (FP32 / BF16: at the contour stencil, in mid; FP64:
            // the field planes of both levels), and both levels are
            // accumulated after it, in order
            float *mid = (float *)(ws + q.off_mid);
            for (int64_t m = 0; m < chunk / 2; ++m) {
                const int64_t n = n0 + 2 * m;
                void *dst = ws + q.off_state[(n0 + m + 1) & 1];
                hipError_t e;
                if (f64) {
                    double *fl1 = which == 1 ? (double *)fields_ptr(q, ws, n + 1) : nullptr;
                    double *fl2 = which == 1 ? (double *)fields_ptr(q, ws, n + 2) : nullptr;
                    e = launch_step2_f64(L, (const double *)(ws + q.off_state[(n0 + m) & 1]), (double *)dst,
                                         incident(q, n), incident(q, n + 1), fl1, fl2, s, two);
                    if (e == hipSuccess && which == 1) e = launch_contour(q.prob.precision, L, fl1, C, s);
                    if (e == hipSuccess && which == 1) e = launch_contour(q.prob.precision, L, fl2, C, s);
                } else {
                    e = launch_step2_neq(q.prob.precision, L, ws + q.off_state[(n0 + m) & 1], dst, incident(q, n),
                                         incident(q, n + 1), which == 1 ? mid : nullptr, s, two);
                    if (e == hipSuccess && which == 1) e = launch_contour2(L, mid, dst, C, s);
                }
                if (e != hipSuccess) {
                    hipGraph_t dummy;
                    (void)hipStreamEndCapture(s, &dummy);
                    return fail(JLB_E_DEVICE, "two-step launch: %s", hipGetErrorString(e));
                }
            }
        } else {
            for (int64_t k = 0; k < chunk; ++k) {
                // FP64 writes field planes only where they are read: the
                // window, and the chunk's last level when the plateau is checked
                int r = launch_one_step(q, ws, L, C, n0 + k, which == 1, plateau && k == chunk - 1,
                                        incident(q, n0 + k), s);
                if (r) {
                    hipGraph_t dummy;
                    (void)hipStreamEndCapture(s, &dummy);
                    return r;
                }
            }
        }
        HIP_TRY(hipStreamEndCapture(s, &g));
        HIP_TRY(hipGraphInstantiate(&gexec[which], g, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(g));
        gstart[which] = n0;
        return JLB_OK;
    };

    int64_t n = 0;
    int64_t passes = 0;
    int graph_used = 0;
    double *dft = (double *)(ws + q.off_dft);
    while (n < steps && rc == JLB_OK) {
        const bool in_window = n >= wstart;
        // chunk must not straddle the window start; the far field's last
        // period runs as single launches, each followed by its phasor terms
        const int64_t far_start = far.s2 ? steps - q.T : steps;
        const int64_t seg_end = std::min(in_window ? steps : wstart, far_start);
        if (use_graph && n >= ramp_end && n + chunk <= seg_end) {
            const int which = in_window ? 1 : 0;
            if (!gexec[which]) {
                rc = capture(which, n);
                if (rc) break;
            }
            // the captured source values repeat with the period after the ramp
            if ((n - gstart[which]) % chunk != 0) {
                rc = fail(JLB_E_DEVICE, "internal: graph phase mismatch");
                break;
            }
            hipError_t e = events && which == 0 && main_launches == 0 ? hipEventRecord(evm0, s) : hipSuccess;
            if (e == hipSuccess) e = hipGraphLaunch(gexec[which], s);
            if (e == hipSuccess && events && which == 0) e = hipEventRecord(evm1, s);
            if (e != hipSuccess) {
                rc = fail(JLB_E_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
                break;
            }
            if (which == 0) main_launches += main_per_chunk;
            graph_used = 1;
            passes += multi >= 0 ? chunk / depth : two_in(which) ? chunk / 2 : chunk;
            n += chunk;
            if (!in_window && check_level(n)) rc = plateau_check(n);
            continue;
        }
        // outside the window with no per-step output (the ramp, the steps
        // before the first whole chunk of the window): multi-step launches
        // in pairs, which leave state n + 2 S in buffer n % 2 as single steps do
        const int64_t pair_end = n < ramp_end ? std::min(ramp_end, seg_end) : seg_end;
        if (multi >= 0 && !in_window && !plateau && !energy && !far.force && n + 2 * depth <= pair_end) {
            for (int k = 0; k < 2 && rc == JLB_OK; ++k) {
                const int64_t m = n + k * depth;
                double einc[4];
                for (int j = 0; j < depth; ++j) einc[j] = incident(q, m + j);
                hipError_t e = launch_stepm_neq(q.prob.precision, L, ws + q.off_state[(n + k) & 1],
                                                ws + q.off_state[(n + k + 1) & 1], einc, nullptr, 0, s, multi);
                if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "multi-step launch: %s", hipGetErrorString(e));
            }
            passes += 2;
            n += 2 * depth;
            continue;
        }
        const bool check = !in_window && check_level(n + 1);
        rc = launch_one_step(q, ws, L, C, n, in_window, energy != nullptr || far.force != nullptr || n == steps - 1 || check,
                             incident(q, n), s);
        if (rc) break;
        ++passes;
        if (check) {
            rc = plateau_check(n + 1);
            if (rc) break;
        }
        if (energy) {
            hipError_t e = launch_energy(q.prob.precision, L, fields_ptr(q, ws, n + 1), (double *)(ws + q.off_parts),
                                         q.nparts, energy + n, s);
            if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "energy launch: %s", hipGetErrorString(e));
        }
        if (far.force && rc == JLB_OK) {
            const double f0 = M_PI * q.prob.radius * q.prob.e0 * q.prob.e0 / 4.0;
            hipError_t e = launch_force_now(q.prob.precision, L, fields_ptr(q, ws, n + 1), C, f0, 2.0 * f0 * q.prob.radius,
                                            far.force + 3 * n, s);
            if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "force trace launch: %s", hipGetErrorString(e));
        }
        if (far.s2 && n >= far_start && rc == JLB_OK) {
            // level n + 1 is inside the window (window >= T), so its fields are in place
            const double ph = 2.0 * M_PI * (double)((n + 1) % q.T) / (double)q.T;
            hipError_t e = launch_far_dft(q.prob.precision, L, fields_ptr(q, ws, n + 1), C, dft, std::cos(ph),
                                          std::sin(ph), s);
            if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "far-field phasor launch: %s", hipGetErrorString(e));
        }
        ++n;
    }
    if (rc == JLB_OK) {
        hipError_t e = events ? hipEventRecord(ev1, s) : hipSuccess;
        if (e == hipSuccess) e = launch_reduce(C, 1.0 / (double)q.window, M_PI * q.prob.radius * q.prob.e0 * q.prob.e0 / 4.0,
                                               2.0 * (M_PI * q.prob.radius * q.prob.e0 * q.prob.e0 / 4.0) * q.prob.radius,
                                               (double *)(ws + q.off_out), s);
        if (e == hipSuccess && far.s2)
            e = launch_far_field(C, dft, 2.0 * M_PI / q.prob.wavelength, 2.0 / (double)q.T, far.nphi, far.s2, s);
        if (e == hipSuccess && ez && hx && hy)
            e = launch_fields_out(q.prob.precision, L, fields_ptr(q, ws, steps), ez, hx, hy, s);
        if (e == hipSuccess)
            e = launch_energy(q.prob.precision, L, fields_ptr(q, ws, steps), (double *)(ws + q.off_parts), q.nparts,
                              (double *)(ws + q.off_out) + 6, s);
        double out[8] = {0};
        if (e == hipSuccess) e = hipMemcpyAsync(out, ws + q.off_out, 7 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "finishing the solve: %s", hipGetErrorString(e));
        if (rc == JLB_OK) {
            float ms = 0.0f;
            if (events) (void)hipEventElapsedTime(&ms, ev0, ev1);
            else ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - loop_t0).count();
            res->fx = out[0];
            res->fy = out[1];
            res->tz = out[2];
            res->fx_raw = out[3];
            res->fy_raw = out[4];
            res->tz_raw = out[5];
            res->loop_ms = ms;
            res->steps_done = steps;
            res->window_steps = q.window;
            res->contour_points = q.nc;
            res->graph_used = graph_used;
            res->bytes_per_step = (int64_t)q.bytes_per_lup * q.nx * q.ny;
            res->state_passes = passes;
            res->energy_final = out[6];
            if (events && main_launches > 0 && !(q.prob.plateau_tol > 0.0)) {
                float mms = 0.0f;
                (void)hipEventElapsedTime(&mms, evm0, evm1);
                res->main_ms = mms;
                res->main_launches = main_launches;
                res->main_kind = main_kind;
                res->main_variant = main_variant;
            }
            for (int k = 0; k < 6; ++k)
                if (!std::isfinite(out[k])) rc = fail(JLB_E_NONFINITE, "forces are not finite");
        }
    } else {
        (void)hipStreamSynchronize(s);
    }
    for (auto &g : gexec)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t ev : {ev0, ev1, evm0, evm1})
        if (ev) (void)hipEventDestroy(ev);
    res->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

// Orders work on the library's stream after the caller's stream, and back.
struct StreamJoin {
    hipStream_t caller, own;
    hipEvent_t ev = nullptr;
    int begin()
    {
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, caller));
        HIP_TRY(hipStreamWaitEvent(own, ev, 0));
        return JLB_OK;
    }
    int end()
    {
        HIP_TRY(hipEventRecord(ev, own));
        HIP_TRY(hipStreamWaitEvent(caller, ev, 0));
        return JLB_OK;
    }
    ~StreamJoin()
    {
        if (ev) (void)hipEventDestroy(ev);
    }
};

}  // namespace jlb

using namespace jlb;

extern "C" {

int jlb_version(void) { return 10000; }

const char *jlb_last_error(void) { return jlb::last_error(); }

int jlb_validate(const jlb_problem *prob)
{
    clear_error();
    Plan q;
    return make_plan(prob, &q);
}

int jlb_workspace_size(const jlb_problem *prob, size_t *bytes)
{
    clear_error();
    if (!bytes) return fail(JLB_E_ARG, "null bytes");
    Plan q;
    int rc = make_plan(prob, &q);
    if (rc) return rc;
    *bytes = q.ws_bytes;
    return JLB_OK;
}

int jlb_material_map(const jlb_problem *prob, uint8_t *mat)
{
    clear_error();
    if (!mat) return fail(JLB_E_ARG, "null mat");
    Plan q;
    int rc = make_plan(prob, &q);
    if (rc) return rc;
    material_map(q, mat, (size_t)q.nx);
    return JLB_OK;
}

static int solve_entry(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res, double *ez,
                       double *hx, double *hy, double *energy, void *stream, FarOut far)
{
    clear_error();
    if (!res) return fail(JLB_E_ARG, "null result");
    Plan q;
    int rc = make_plan(prob, &q);
    if (rc) return rc;
    if ((ez || hx || hy) && !(ez && hx && hy)) return fail(JLB_E_ARG, "ez, hx, hy must all be given or all NULL");
    if (workspace && workspace_bytes < q.ws_bytes)
        return fail(JLB_E_OOM, "workspace %zu bytes < %zu needed", workspace_bytes, q.ws_bytes);
    hipStream_t own = own_stream();
    if (!own) return fail(JLB_E_DEVICE, "cannot create a stream");
    StreamJoin join{(hipStream_t)stream, own};
    rc = join.begin();
    if (rc) return rc;
    char *ws = (char *)workspace;
    bool owned = false;
    if (!ws) {
        hipError_t e = hipMalloc((void **)&ws, q.ws_bytes);
        if (e != hipSuccess) return fail(JLB_E_OOM, "hipMalloc(%zu): %s", q.ws_bytes, hipGetErrorString(e));
        owned = true;
    }
    rc = run_solve(q, ws, res, ez, hx, hy, energy, own, far);
    int rc2 = join.end();
    if (owned) {
        (void)hipStreamSynchronize(own);
        (void)hipFree(ws);
    }
    return rc ? rc : rc2;
}

int jlb_solve(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res, double *ez,
              double *hx, double *hy, double *energy, void *stream)
{
    return solve_entry(prob, workspace, workspace_bytes, res, ez, hx, hy, energy, stream, FarOut{0, nullptr});
}

int jlb_solve_force_trace(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res,
                          double *force, void *stream)
{
    clear_error();
    if (!force) return fail(JLB_E_ARG, "null force");
    return solve_entry(prob, workspace, workspace_bytes, res, nullptr, nullptr, nullptr, nullptr, stream,
                       FarOut{0, nullptr, force});
}

int jlb_solve_far_field(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res,
                        int32_t n_angles, double *s2, void *stream)
{
    clear_error();
    if (!s2) return fail(JLB_E_ARG, "null s2");
    if (n_angles < 1 || n_angles > JLB_MAX_FAR_ANGLES)
        return fail(JLB_E_ARG, "n_angles %d outside 1..%d", n_angles, JLB_MAX_FAR_ANGLES);
    return solve_entry(prob, workspace, workspace_bytes, res, nullptr, nullptr, nullptr, nullptr, stream,
                       FarOut{n_angles, s2});
}

int jlb_solve_static(const jlb_problem *prob, jlb_result *res, double *ez, double *hx, double *hy, void *stream)
{
    clear_error();
    if (!res) return fail(JLB_E_ARG, "null result");
    Plan q;
    int rc = make_plan(prob, &q);
    if (rc) return rc;
    if ((ez || hx || hy) && !(ez && hx && hy)) return fail(JLB_E_ARG, "ez, hx, hy must all be given or all NULL");
    if (q.prob.plateau_tol > 0.0) return fail(JLB_E_ARG, "jlb_solve_static has no plateau stop");
    if (q.ws_bytes > JLB_STATIC_SCRATCH_BYTES)
        return fail(JLB_E_OOM, "problem needs %zu bytes of scratch, more than the library-held %zu (use jlb_solve)",
                    q.ws_bytes, (size_t)JLB_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    hipError_t e = static_scratch(&ws);
    if (e != hipSuccess) return fail(JLB_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
    // direct launches on the caller's stream: no graph, no stream or event of
    // the library's own
    q.prob.flags |= JLB_F_NO_GRAPH;
    return run_solve(q, (char *)ws, res, ez, hx, hy, nullptr, (hipStream_t)stream, FarOut{0, nullptr}, false);
}

// kind: 1 single-step, 2 two-step, 3 multi-step variant
static int time_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                            int32_t launches, int variant, int kind, double *ms_per_launch, void *stream)
{
    if (!ms_per_launch || launches < 1 || warmup < 0) return fail(JLB_E_ARG, "bad launch counts");
    Plan q;
    int rc = make_plan(prob, &q);
    if (rc) return rc;
    if (workspace && workspace_bytes < q.ws_bytes) return fail(JLB_E_OOM, "workspace too small");
    hipStream_t own = own_stream();
    if (!own) return fail(JLB_E_DEVICE, "cannot create a stream");
    StreamJoin join{(hipStream_t)stream, own};
    rc = join.begin();
    if (rc) return rc;
    char *ws = (char *)workspace;
    bool owned = false;
    if (!ws) {
        if (hipMalloc((void **)&ws, q.ws_bytes) != hipSuccess) return fail(JLB_E_OOM, "hipMalloc failed");
        owned = true;
    }
    rc = upload_setup(q, ws, own);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == JLB_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(JLB_E_DEVICE, "event create");
    const Lattice L = lattice_of(q, (const uint8_t *)(ws + q.off_mask));
    // warm-up launches directly, then the timed launches captured into a
    // hipGraph and replayed (once to warm it, once timed), as a solve runs them
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    for (int64_t n = 0; rc == JLB_OK && n < (int64_t)warmup + launches; ++n) {
        if (n == warmup && hipStreamBeginCapture(own, hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = fail(JLB_E_DEVICE, "capture begin");
        if (rc) break;
        void *src = ws + q.off_state[n & 1], *dst = ws + q.off_state[(n + 1) & 1];
        hipError_t e;
        if (kind == 3) {
            int depth = 0, rows = 0;
            multi_step_shape(variant, depth, rows);
            double einc[4];
            for (int k = 0; k < depth; ++k) einc[k] = incident(q, depth * n + k);
            e = launch_stepm_neq(q.prob.precision, L, src, dst, einc, nullptr, 0, own, variant);
        } else if (kind == 2) {
            e = q.prob.precision == JLB_FP64
                    ? launch_step2_f64(L, (const double *)src, (double *)dst, incident(q, 2 * n), incident(q, 2 * n + 1),
                                       nullptr, nullptr, own, variant)
                    : launch_step2_neq(q.prob.precision, L, src, dst, incident(q, 2 * n), incident(q, 2 * n + 1),
                                       nullptr, own, variant);
        } else {
            e = launch_step(q, L, src, dst, nullptr, incident(q, n), own, variant);
        }
        if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "step launch: %s", hipGetErrorString(e));
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(own, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone) {
        if (hipStreamEndCapture(own, &graph) != hipSuccess && rc == JLB_OK) rc = fail(JLB_E_DEVICE, "capture end");
    }
    if (rc == JLB_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(JLB_E_DEVICE, "graph instantiate");
    if (rc == JLB_OK) {
        float ms = 0.0f;
        if (hipGraphLaunch(exec, own) != hipSuccess || hipEventRecord(e0, own) != hipSuccess ||
            hipGraphLaunch(exec, own) != hipSuccess || hipEventRecord(e1, own) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = fail(JLB_E_DEVICE, "event timing");
        *ms_per_launch = (double)ms / launches;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    int rc2 = join.end();
    (void)hipStreamSynchronize(own);
    if (owned) (void)hipFree(ws);
    return rc ? rc : rc2;
}

int jlb_time_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                         int32_t launches, double *ms_per_launch, void *stream)
{
    clear_error();
    if (!prob) return fail(JLB_E_ARG, "null problem");
    const int v = prob->precision >= 0 && prob->precision <= 2 ? step_variant(prob->precision) : 0;
    return time_step_kernel(prob, workspace, workspace_bytes, warmup, launches, v, 1, ms_per_launch, stream);
}

int jlb_time_two_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                             int32_t launches, double *ms_per_launch, void *stream)
{
    clear_error();
    if (!prob) return fail(JLB_E_ARG, "null problem");
    if (prob->precision < 0 || prob->precision > 2) return fail(JLB_E_ARG, "unknown precision");
    const int v = two_step_variant(prob->precision);
    if (v < 0) return fail(JLB_E_ARG, "no two-step variant selected");
    return time_step_kernel(prob, workspace, workspace_bytes, warmup, launches, v, 2, ms_per_launch, stream);
}

int jlb_time_multi_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                               int32_t launches, double *ms_per_launch, void *stream)
{
    clear_error();
    if (!prob) return fail(JLB_E_ARG, "null problem");
    if (prob->precision != JLB_FP32 && prob->precision != JLB_BF16)
        return fail(JLB_E_ARG, "multi-step kernels are FP32 / BF16");
    const int v = multi_step_variant(prob->precision);
    if (v < 0) return fail(JLB_E_ARG, "no multi-step variant selected");
    int depth = 0, rows = 0;
    multi_step_shape(v, depth, rows);
    if (prob->ny < rows + depth) return fail(JLB_E_ARG, "grid too short for this multi-step variant");
    return time_step_kernel(prob, workspace, workspace_bytes, warmup, launches, v, 3, ms_per_launch, stream);
}

int jlb_multi_step_shape(int32_t variant, int32_t *depth, int32_t *rows)
{
    clear_error();
    if (variant < 0 || variant >= MULTI_STEP_VARIANTS || !depth || !rows)
        return fail(JLB_E_ARG, "variant 0..%d and non-null outputs", MULTI_STEP_VARIANTS - 1);
    int d = 0, r = 0;
    multi_step_shape(variant, d, r);
    *depth = d;
    *rows = r;
    return JLB_OK;
}

int jlb_autotune(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t launches,
                 int32_t *best_variant, double *ms_per_variant, void *stream)
{
    clear_error();
    if (!prob || !best_variant) return fail(JLB_E_ARG, "null argument");
    if (launches < 1) return fail(JLB_E_ARG, "launches must be >= 1");
    const int nvar = prob->precision == JLB_FP64 ? F64_VARIANTS : NEQ_VARIANTS;
    double best = 1e300;
    int bv = step_variant(prob->precision);
    for (int v = 0; v < nvar; ++v) {
        double ms = 0.0;
        int rc = time_step_kernel(prob, workspace, workspace_bytes, 2, launches, v, 1, &ms, stream);
        if (rc) return rc;
        if (ms_per_variant) ms_per_variant[v] = ms;
        if (ms < best) {
            best = ms;
            bv = v;
        }
    }
    set_step_variant(prob->precision, bv);
    *best_variant = bv;
    if (prob->precision == JLB_FP64) {
        // FP64 two-step kernels, compared per lattice step
        int b2 = -1;
        for (int v = 0; v < F64_TWO_STEP_VARIANTS; ++v) {
            double ms = 0.0;
            int rc = time_step_kernel(prob, workspace, workspace_bytes, 2, launches, v, 2, &ms, stream);
            if (rc) return rc;
            ms *= 0.5;
            if (ms_per_variant) ms_per_variant[F64_VARIANTS + v] = ms;
            if (ms < best) {
                best = ms;
                b2 = v;
            }
        }
        set_two_step_variant(prob->precision, b2);
        if (b2 >= 0) *best_variant = F64_VARIANTS + b2;
        return JLB_OK;
    }
    // two-step kernels, compared per lattice step
    int b2 = -1;
    for (int v = 0; v < TWO_STEP_VARIANTS; ++v) {
        double ms = 0.0;
        int rc = time_step_kernel(prob, workspace, workspace_bytes, 2, launches, v, 2, &ms, stream);
        if (rc) return rc;
        ms *= 0.5;
        if (ms_per_variant) ms_per_variant[NEQ_VARIANTS + v] = ms;
        if (ms < best) {
            best = ms;
            b2 = v;
        }
    }
    set_two_step_variant(prob->precision, b2);
    if (b2 >= 0) *best_variant = NEQ_VARIANTS + b2;
    // multi-step kernels (the periods before the window), per lattice step,
    // against the best of the above; variants the grid is too short for are
    // skipped (their entry stays 0)
    int bm = -1;
    for (int v = 0; v < MULTI_STEP_VARIANTS; ++v) {
        if (ms_per_variant) ms_per_variant[NEQ_VARIANTS + TWO_STEP_VARIANTS + v] = 0.0;
        int depth = 0, rows = 0;
        multi_step_shape(v, depth, rows);
        if (prob->ny < rows + depth) continue;
        double ms = 0.0;
        int rc = time_step_kernel(prob, workspace, workspace_bytes, 2, launches, v, 3, &ms, stream);
        if (rc) return rc;
        ms /= depth;
        if (ms_per_variant) ms_per_variant[NEQ_VARIANTS + TWO_STEP_VARIANTS + v] = ms;
        // a three-step variant has to win by 3 %: over a whole solve its extra
        // state passes and launches cost more than this short timing shows
        // (1024^2: three-step H7 timed within 1 % of four-step H10 ran 10 %
        // slower in the solve)
        const double score = depth == 3 ? 1.03 * ms : ms;
        if (score < best) {
            best = score;
            bm = v;
        }
    }
    set_multi_step_variant(prob->precision, bm);
    return JLB_OK;
}

int jlb_set_step_variant(int32_t precision, int32_t variant)
{
    clear_error();
    const int nvar = precision == JLB_FP64 ? F64_VARIANTS : NEQ_VARIANTS;
    if (precision < 0 || precision > 2 || variant < 0 || variant >= nvar)
        return fail(JLB_E_ARG, "precision 0..2 and variant 0..%d", nvar - 1);
    set_step_variant(precision, variant);
    return JLB_OK;
}

int jlb_set_two_step_variant(int32_t precision, int32_t variant)
{
    clear_error();
    const int nvar = precision == JLB_FP64 ? F64_TWO_STEP_VARIANTS : TWO_STEP_VARIANTS;
    if (precision < 0 || precision > 2 || variant < -1 || variant >= nvar)
        return fail(JLB_E_ARG, "precision 0..2 and variant -1..%d", nvar - 1);
    set_two_step_variant(precision, variant);
    return JLB_OK;
}

int jlb_set_multi_step_variant(int32_t precision, int32_t variant)
{
    clear_error();
    if (precision < 0 || precision > 2 || variant < -1 || variant >= MULTI_STEP_VARIANTS ||
        (precision == JLB_FP64 && variant != -1))
        return fail(JLB_E_ARG, "precision 1..2 and variant -1..%d (FP64: -1 only)", MULTI_STEP_VARIANTS - 1);
    set_multi_step_variant(precision, variant);
    return JLB_OK;
}

int jlb_get_multi_step_variant(int32_t precision, int32_t *variant)
{
    clear_error();
    if (precision < 0 || precision > 2 || !variant) return fail(JLB_E_ARG, "bad precision or null variant");
    *variant = multi_step_variant(precision);
    return JLB_OK;
}

int jlb_get_two_step_variant(int32_t precision, int32_t *variant)
{
    clear_error();
    if (precision < 0 || precision > 2 || !variant) return fail(JLB_E_ARG, "bad precision or null variant");
    *variant = two_step_variant(precision);
    return JLB_OK;
}

int jlb_get_step_variant(int32_t precision, int32_t *variant)
{
    clear_error();
    if (precision < 0 || precision > 2 || !variant) return fail(JLB_E_ARG, "bad precision or null variant");
    *variant = step_variant(precision);
    return JLB_OK;
}

int jlb_copy_bandwidth(size_t bytes, int32_t launches, double *ms_per_launch, void *stream)
{
    clear_error();
    if (!ms_per_launch || launches < 1 || bytes < 16) return fail(JLB_E_ARG, "bad copy arguments");
    bytes &= ~(size_t)15;
    hipStream_t own = own_stream();
    if (!own) return fail(JLB_E_DEVICE, "cannot create a stream");
    StreamJoin join{(hipStream_t)stream, own};
    int rc = join.begin();
    if (rc) return rc;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        if (a) (void)hipFree(a);
        return fail(JLB_E_OOM, "copy buffers of %zu bytes", bytes);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemsetAsync(a, 0, bytes, own);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_copy(a, b, bytes, own);
    if (e == hipSuccess) e = hipEventRecord(e0, own);
    for (int k = 0; k < launches && e == hipSuccess; ++k) e = launch_copy(a, b, bytes, own);
    if (e == hipSuccess) e = hipEventRecord(e1, own);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = fail(JLB_E_DEVICE, "copy timing: %s", hipGetErrorString(e));
    else *ms_per_launch = (double)ms / launches;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    int rc2 = join.end();
    return rc ? rc : rc2;
}

}  // extern "C"
