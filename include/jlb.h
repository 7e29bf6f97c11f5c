/*
 * jlb.h -- C ABI of the MI355X (gfx950) library for the electromagnetic
 * lattice Boltzmann solve of TM^z plane-wave scattering off a circular Janus
 * cylinder and the radiation force and torque that follow from it.
 *
 * Method (arXiv 2509.22308):
 *   Sec. II, Fig. (schematic)   cylinder of radius a at the domain centre,
 *                               split by a diameter into region II (eps_r1)
 *                               and region III (PEC or eps_r2), vacuum outside;
 *                               plane wave entering from the left, interface
 *                               angle phi0.
 *   Sec. III, Eqs. (LBGK equation), (equilibrium distribution functions)
 *                               D3Q7 electric and magnetic populations,
 *                               tau = 1/2 update f -> 2 f^eq - f, fields as
 *                               moments, per-cell permittivity, mu_r = 1;
 *                               a perfect conductor (E_z^tot = 0, Sec. II)
 *                               is a node whose electric field is zero, the
 *                               update's limit of infinite permittivity.
 *   Sec. II.B, Eqs. (stress tensor average), (force), (torque)
 *                               time-averaged Maxwell stress on a closed
 *                               contour around the body -> F_x, F_y, M_z,
 *                               normalised by F0 = pi a eps0 E0^2 / 4 and
 *                               M0 = 2 F0 a.
 *
 * Lattice units: dx = dt = 1, eps0 = mu0 = 1.  The model's vacuum wave speed
 * is 1/3 cell per step, so the angular frequency is omega = 2 pi / (3 lambda)
 * and the period is T = 3 lambda steps; 3 lambda must be an integer.
 *
 * Conventions shared by every call:
 *   - every function returns int: JLB_OK (0) or a negative JLB_E_* code; the
 *     calling thread's jlb_last_error() then describes the failure;
 *   - no C++ exception crosses this boundary;
 *   - 2-D arrays are row-major [ny][nx] with x (the direction of incidence)
 *     fastest;
 *   - "device" pointers are HIP device allocations on the current device,
 *     "host" pointers ordinary host memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls order their work after prior work on it and return only when
 *     their results are complete (the solve is synchronous for the host).
 */
#ifndef JLB_H
#define JLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JLB_OK 0
#define JLB_E_ARG -1          /* a parameter is out of range or a pointer is missing          */
#define JLB_E_GEOMETRY -2     /* disk + contour + margin do not fit inside the domain         */
#define JLB_E_RESOLUTION -3   /* lambda / sqrt(eps_max) < 10 (Sec. III) without the override  */
#define JLB_E_WINDOW -4       /* steps < (avg_periods + ramp_periods) * T                      */
#define JLB_E_OOM -5          /* workspace too small or device allocation failed              */
#define JLB_E_DEVICE -6       /* a HIP runtime call failed                                     */
#define JLB_E_NONFINITE -7    /* the forces came out NaN or infinite                           */
#define JLB_E_ADMISSION -8    /* engine: the request can never fit the engine's memory budget */
#define JLB_E_STATE -9        /* engine: unknown ticket or call out of order                   */

/* Sec. II: body kinds. */
typedef enum {
    JLB_HOMOGENEOUS = 0,              /* whole disk eps1                                  */
    JLB_DIELECTRIC_JANUS = 1,         /* region II eps1, region III eps2                  */
    JLB_METALLO_DIELECTRIC_JANUS = 2  /* region II eps1, region III perfect conductor     */
} jlb_kind;

/* Storage and arithmetic of the populations. */
typedef enum {
    JLB_FP64 = 0,  /* 11 populations per cell in FP64, FP64 arithmetic            */
    JLB_FP32 = 1,  /* fields (Ez, Hx, Hy) in FP32 + 8 moving-population deviations
                      from equilibrium in FP32; FP32 arithmetic                    */
    JLB_BF16 = 2   /* as JLB_FP32 but the 8 deviations stored in bfloat16         */
} jlb_precision;

/* jlb_problem.flags */
#define JLB_F_ALLOW_UNDERRESOLVED 1u  /* skip the lambda / sqrt(eps_max) >= 10 check         */
#define JLB_F_NO_GRAPH 2u             /* launch every step directly instead of replaying a
                                         captured hipGraph of whole periods                  */
#define JLB_F_CENTRE 4u               /* place the disk centre at (cx, cy) (node coordinates)
                                         instead of the grid centre ((nx-1)/2, (ny-1)/2)  */

/*
 * One scattering problem (Sec. II; Sec. III for the domain and the source).
 * The cylinder centre is ((nx-1)/2, (ny-1)/2) in node coordinates.  A node
 * (i, j) with d = (i - cx, j - cy) is inside when |d|^2 <= a^2; inside nodes
 * with d . (-sin phi0, -cos phi0) > 1e-9 are region II, the rest region III.
 * With this lab frame phi0 = pi/2 puts region II towards the incoming wave
 * and phi0 = 0 puts region III on the +y side, as in Sec. IV.A and App. A.
 */
typedef struct {
    int32_t nx, ny;          /* grid nodes, each >= 16                                    */
    int32_t kind;            /* jlb_kind                                                  */
    int32_t precision;       /* jlb_precision                                             */
    double radius;           /* a, cells, > 0                                             */
    double eps1, eps2;       /* relative permittivities of regions II and III, >= 1      */
    double phi0;             /* interface angle, radians                                  */
    double wavelength;       /* lambda, cells; 3 * lambda integer                         */
    double e0;               /* incident amplitude E0 (> 0)                               */
    int64_t steps;           /* lattice time steps                                        */
    int32_t avg_periods;     /* average the stress over the last avg_periods * T steps    */
    int32_t ramp_periods;    /* raised-cosine source ramp length in periods (>= 0)        */
    double contour_offset;   /* contour radius R_c = radius + contour_offset (> 0)        */
    int32_t contour_points;  /* samples on the contour; 0 selects 8 * ceil(2 pi R_c / 8)  */
    uint32_t flags;          /* JLB_F_*                                                   */
    double plateau_tol;      /* > 0: plateau stop (jlb_solve only; see below); 0: off     */
    int32_t polarization;    /* JLB_TM (0, Sec. II) or JLB_TE (1; see below)               */
    int32_t reserved;        /* 0                                                         */
    double cx, cy;           /* disk centre in node coordinates, with JLB_F_CENTRE         */
} jlb_problem;

/*
 * Polarisation.  JLB_TM: Ez, Hx, Hy (the paper's case throughout).  JLB_TE:
 * Hz, Ex, Ey, the case the paper leaves for later work (Sec. I), on the same
 * lattice and printed update (Sec. III, Eqs. LBGK equation and equilibrium
 * distribution functions) with the incident wave Ey = Hz = E_inc travelling
 * +x; forces use the same stress (Sec. II.B) and normalisation.  For TE the
 * field outputs of jlb_solve (ez, hx, hy) hold Hz, Ex, Ey, and the far field
 * of jlb_solve_far_field is k0 r |Hz^S|^2 / |Hz^I|^2.  Every kernel, the
 * two-step ones included, runs both polarisations.
 */
#define JLB_TM 0
#define JLB_TE 1

/*
 * Plateau stop (Sec. III: convergence is judged by the total field energy
 * approaching a constant).  With plateau_tol > 0, jlb_solve samples the
 * energy W = sum over the non-conductor nodes of (eps Ez^2 + Hx^2 + Hy^2)/2
 * at fixed-phase check points: the end of the ramp (L0 = ramp_periods T) and
 * every P_c steps after it, P_c = T, 2T or 4T (the shortest whole number of
 * periods that is a multiple of 4 steps).  At the first check point L >= L0 +
 * 2 P_c with |W(L) - W(L - P_c)| <= plateau_tol W(L) and L + avg_periods T <=
 * steps, the solve averages the levels L + 1 .. L + avg_periods T and stops
 * there (jlb_result.steps_done); without such a point it is the plain solve.
 * The engine rejects it (JLB_E_ARG): its solves run their full step count.
 */

/* Outcome of one solve (host struct, written by the library). */
typedef struct {
    double fx, fy, tz;              /* F~x, F~y, M~z (Sec. II.B normalisation)                */
    double fx_raw, fy_raw, tz_raw;  /* per unit length in lattice units                       */
    double loop_ms;                 /* HIP-event time of the time-stepping loop on the device */
    double total_ms;                /* host wall time of the whole call                       */
    int64_t steps_done;
    int64_t window_steps;           /* time samples in the stress average                     */
    int32_t contour_points;
    int32_t graph_used;             /* 1 when whole periods were replayed from a hipGraph     */
    int64_t bytes_per_step;         /* algorithmic HBM bytes of one pass over the state        */
    int64_t state_passes;           /* step-kernel launches (a two-step launch is one pass)    */
    double energy_final;            /* field energy sum (eps E^2 + H^2)/2 after the last step  */
    /* The whole periods before the window replayed from a hipGraph (the bulk
       of a long solve): HIP-event time on the solve's stream, step-kernel
       launches in it, and which kernel ran there: main_kind 1 single step
       (main_variant: step variant), 2 two-step, 3 multi-step; 0 when no such
       stretch ran (jlb_solve only; the engine leaves these 0). */
    double main_ms;
    int64_t main_launches;
    int32_t main_kind, main_variant;
} jlb_result;

/* Library version (major * 10000 + minor * 100 + patch). */
int jlb_version(void);

/* Description of the last failure on the calling thread ("" if none). */
const char *jlb_last_error(void);

/*
 * Checks a problem without touching the device: argument ranges, geometry
 * (disk, contour and a 4-cell margin inside the grid, contour outside the
 * disk), resolution (Sec. III: lambda / sqrt(eps_max) >= 10 unless
 * JLB_F_ALLOW_UNDERRESOLVED) and the averaging window.  Returns JLB_OK or the
 * JLB_E_* code of the first violation.
 */
int jlb_validate(const jlb_problem *prob);

/*
 * Device workspace one solve of `prob` needs, in bytes (host out-pointer).
 * The grid carries one extra row for the incident-wave companion lattice and
 * pads rows to a multiple of 16 nodes.
 */
int jlb_workspace_size(const jlb_problem *prob, size_t *bytes);

/*
 * Material map of `prob` (Sec. II geometry; staircase on the nodes) into the
 * caller's host array mat[ny][nx]: 0 vacuum, 1 region II, 2 region III
 * dielectric, 3 perfect conductor.
 */
int jlb_material_map(const jlb_problem *prob, uint8_t *mat);

/*
 * Runs one solve on the device (Sec. III time stepping, Sec. II.B stress
 * average and contour integral) and writes the forces to *res (host).
 *   workspace        device buffer of at least jlb_workspace_size() bytes,
 *                    owned by the caller and not used by others during the
 *                    call; NULL makes the library allocate and free its own
 *   ez, hx, hy       optional device arrays [ny][nx] of double: the fields
 *                    after the last step (zero on conductor nodes), written
 *                    in FP64 whatever the storage precision; NULL to skip
 *   energy           optional device array [steps] of double: the field
 *                    energy sum (eps Ez^2 + Hx^2 + Hy^2)/2 after each step;
 *                    NULL to skip (tracing slows the solve)
 * Errors: any code of jlb_validate, JLB_E_OOM, JLB_E_DEVICE, and
 * JLB_E_NONFINITE when the forces are not finite (e.g. an unstable setup).
 */
int jlb_solve(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res,
              double *ez, double *hx, double *hy, double *energy, void *stream);

/*
 * Instantaneous force trace (Sec. III: the forces settle into a steady
 * oscillation at twice the frequency of the incident wave).  The solve of
 * jlb_solve (same result), and after every step n the stress integral of
 * Sec. II.B evaluated with the fields of level n + 1 instead of their time
 * average, normalised as F~x, F~y, M~z, into the caller's device array
 * force[steps][3] of double.  Over the averaging window the entries average
 * to the result's forces.  Steps are launched one at a time (no graph, no
 * two-step kernels), as with the energy trace; with the plateau stop, rows
 * past jlb_result.steps_done are left untouched.
 * Errors: as jlb_solve; JLB_E_ARG for force NULL.
 */
int jlb_solve_force_trace(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res,
                          double *force, void *stream);

/*
 * Far field (Sec. II.A, Eq. scattering intensity): the solve of jlb_solve
 * (same forces in *res) plus the scattering intensity
 *   |S(phi)|^2 = k0 r |E^S|^2 / |E^I|^2  (r -> infinity)
 * at the lab angles phi_a = 2 pi a / n_angles, a = 0 .. n_angles - 1 (0 is
 * the incident direction +x, angles counter-clockwise), into the caller's
 * device array s2[n_angles] of double.
 * Method: over the last period T of the run (single-step launches) the
 * single-bin phasors (2 / T) sum_t F(t) exp(j omega t) of Ez, Hx, Hy are
 * accumulated in FP64 at the stress contour's samples, together with those
 * of the lattice's own incident wave (the companion row) at the same x;
 * scattered = total - incident (Sec. III).  A near-to-far-field transform on
 * the contour (Green's theorem with the large-argument Hankel form) gives
 *   |S|^2 = k0^2 |I|^2 / (8 pi |E^I|^2),
 *   I(phi) = sum_k w [J_z - (n_k . u) E_z^S] exp(-j k0 u . r_k),
 * J_z = n_x H_y - n_y H_x, u = (cos phi, sin phi), w = 2 pi R_c / N_c,
 * k0 = 2 pi / lambda, |E^I|^2 the mean incident intensity over the samples.
 * Errors: as jlb_solve; JLB_E_ARG for s2 NULL or n_angles outside
 * 1..JLB_MAX_FAR_ANGLES.  The plateau stop applies as in jlb_solve (the
 * phasors then cover the last period before its stop).
 */
#define JLB_MAX_FAR_ANGLES 65536
int jlb_solve_far_field(const jlb_problem *prob, void *workspace, size_t workspace_bytes, jlb_result *res,
                        int32_t n_angles, double *s2, void *stream);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * solve of jlb_solve on a workspace the library holds itself, a file-scope
 * device array of JLB_STATIC_SCRATCH_BYTES bytes per device, created when the
 * library is loaded on that device and kept until the process ends.  The call
 * allocates no device memory and creates no stream, event or graph: every
 * step is a direct launch on `stream`, and the results equal those of
 * jlb_solve bit for bit.
 *   prob             as for jlb_solve (no plateau stop: JLB_E_ARG)
 *   res              host struct; loop_ms is host time, main_* are 0
 *   ez, hx, hy       optional device arrays [ny][nx] of double, as jlb_solve
 *   stream           hipStream_t as void* (NULL = the null stream)
 * The array is shared by every call on a device and keeps the last call's
 * contents; the call clears what must start at zero.  Calls that overlap on
 * one device (other threads, other streams) race on it and must not be made.
 * Errors: as jlb_validate; JLB_E_OOM when jlb_workspace_size(prob) exceeds
 * JLB_STATIC_SCRATCH_BYTES (use jlb_solve then); JLB_E_DEVICE;
 * JLB_E_NONFINITE.
 */
#define JLB_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int jlb_solve_static(const jlb_problem *prob, jlb_result *res, double *ez, double *hx, double *hy, void *stream);

/*
 * Overdamped motion of the cylinder under its radiation force and torque
 * (Sec. IV.C: force and torque balance with the slender-body resistance,
 * giving in t~ = t / T0, T0 = a eta / F0, (x~, y~) = (x, y) / a:
 *   dx~/dt~ = log(l/a) F~x(phi0) / (4 pi),  dy~/dt~ = log(l/a) F~y(phi0) / (4 pi),
 *   dphi0/dt~ = M~z(phi0) / (2 pi)).
 * F~x, F~y, M~z are one row of a design map: host arrays of n >= 4 samples at
 * the uniform angles phi_k = phi_first + 2 pi k / n (one period, no repeated
 * end point), interpolated by the periodic cubic spline through them.  The
 * classical fourth-order Runge-Kutta method with step dt integrates nsteps
 * steps from (0, 0, phi_start).  out (host, caller-owned) receives
 * floor(nsteps / record_every) + 1 rows of (t~, x~, y~, phi0) at steps 0,
 * record_every, 2 record_every, ...; phi0 is not wrapped.  Host only (no
 * device work).  Errors: JLB_E_ARG for n < 4, a NULL array, dt <= 0,
 * nsteps < 0, record_every < 1 or a non-finite input.
 */
int jlb_trajectory(int32_t n, double phi_first, const double *fx, const double *fy, const double *tz,
                   double phi_start, double dt, int64_t nsteps, double log_l_over_a, int32_t record_every,
                   double *out);

/*
 * Times `launches` back-to-back launches of the fused lattice-step kernel
 * of `prob` (no contour work), on `stream`: after `warmup` untimed direct
 * launches, the `launches` launches are captured into a hipGraph, replayed
 * once untimed and once between two HIP events, as a solve replays its
 * periods; *ms_per_launch (host) receives the mean.  The workspace is as
 * for jlb_solve (NULL allocates).  The state starts at zero and the source
 * is on, so the kernel takes the same paths as in a solve.
 */
int jlb_time_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                         int32_t launches, double *ms_per_launch, void *stream);

/*
 * The lattice step has kernel variants with identical results and different
 * thread-to-node mappings.  FP32 / BF16 (JLB_STEP_VARIANTS of them):
 *   0       one node per thread, 64 x 4 node blocks;
 *   1/2     two / four adjacent nodes per thread (two- / four-wide loads and
 *           stores), one row per thread, 64 x 4 thread blocks;
 *   3/4     the same with 256 x 1 thread blocks;  5/6  with 256 x 2.
 * FP64 (JLB_FP64_STEP_VARIANTS): 0 / 1 / 2 one node per thread in 64 x 4 /
 * 256 x 1 / 256 x 2 thread blocks; 3 / 4 two adjacent nodes per thread
 * (16-byte loads and stores) in 64 x 4 / 256 x 1 thread blocks.  The batched
 * engine runs variants 3 and 4 as variant 0.
 * The choice is process-wide per precision (default 0 until jlb_autotune or
 * jlb_set_step_variant picks another).
 *
 * FP32 / BF16 also have two-step kernels (JLB_TWO_STEP_VARIANTS of them):
 * one launch takes the state from step n to n + 2, reading and writing it
 * once (temporal blocking), with results equal to two single steps bit for
 * bit.  When no multi-step variant applies, an FP32 / BF16 solve uses the
 * selected two-step variant for every step that runs in graph-captured whole
 * periods (inside the averaging window too, where the middle level's contour
 * fields are kept), and single steps for the ramp, the steps after the last
 * whole chunk and a far-field solve's last period; the engine uses it for the
 * steps of its FP32 / BF16 solves that its four-step launches do not take.
 * Variants (V adjacent nodes per lane, H rows per wavefront, HX halo columns
 * per side; HX 8 keeps output strips 64-byte aligned; LA2: each input row is
 * loaded two rows ahead of its first use instead of one): 0 V1 H8 X2,
 * 1 V1 H16 X2, 2 V2 H8 X2, 3 V2 H16 X2, 4 V1 H8 X8, 5 V2 H16 X8, 6 V2 H32 X8,
 * 7 V1 H8 X8 LA2, 8 V1 H4 X8 LA2, 9 V1 H16 X8 LA2.  Default: 4 (set -1 for
 * single steps only).
 *
 * FP64 has two-step kernels too (JLB_FP64_TWO_STEP_VARIANTS of them, one
 * node per lane, H rows per wavefront, X4 / X8 halo columns per side (X8:
 * every strip stores whole 128-byte lines, which pays on grids streamed
 * from HBM), registers for two or (W3) three wavefronts per SIMD, LA2 as
 * above): 0 H10 X4, 1 H12 X4, 2 H12 X4 W3, 3 H12 X4 LA2, 4 H6 X8, 5 H8 X8,
 * 6 H8 X8 LA2, 7 H12 X8 (default 0).  An
 * FP64 solve uses the selected one for its graph-captured periods, inside
 * the averaging window too (there it also writes the field planes of both
 * levels), but not with the plateau stop, and single steps elsewhere;
 * results equal single steps bit for bit.  The engine runs its FP64 solves
 * on the selected FP64 two-step variant too (batched over the resident
 * solves), or on single steps when it is -1.
 *
 * jlb_autotune times every single-step variant of prob->precision on prob's
 * grid (`launches` timed launches each, after 2 warm-up launches; workspace
 * as for jlb_solve) and makes the fastest the current choice; it then times
 * the two-step variants and selects the fastest of them when its time per
 * lattice step beats the best single step (else turns two-step kernels off;
 * for FP64 *best_variant is then JLB_FP64_STEP_VARIANTS + the two-step
 * index, and ms_per_variant holds the FP64 two-step times after the
 * single-step ones); for FP32 / BF16 it then times the multi-step variants the grid allows and
 * selects the fastest of them when its time per lattice step beats the best
 * so far (else turns them off); a three-step variant's time counts 3 % more
 * (over a whole solve its extra state passes and launches cost more than the
 * short timing shows).  Timings are graph replays (jlb_time_step_kernel).  *best_variant receives the winner of the
 * first two rounds: a single-step variant index, or JLB_STEP_VARIANTS + the
 * two-step index (jlb_get_multi_step_variant reports the third).
 * ms_per_variant (host, optional) receives the mean time per lattice step in
 * ms, single-step variants first, then the two-step ones, then the
 * multi-step ones, 0 for those not timed (JLB_STEP_VARIANTS +
 * JLB_TWO_STEP_VARIANTS + JLB_MULTI_STEP_VARIANTS entries are always enough).
 */
#define JLB_STEP_VARIANTS 7
#define JLB_FP64_STEP_VARIANTS 5
#define JLB_TWO_STEP_VARIANTS 10
#define JLB_FP64_TWO_STEP_VARIANTS 8
int jlb_autotune(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t launches,
                 int32_t *best_variant, double *ms_per_variant, void *stream);

/* Forces (set) or reports (get) the current FP32 / BF16 step variant. */
int jlb_set_step_variant(int32_t precision, int32_t variant);
/* Forces (set, -1 = off) or reports (get) the current two-step variant. */
int jlb_set_two_step_variant(int32_t precision, int32_t variant);
int jlb_get_two_step_variant(int32_t precision, int32_t *variant);
/*
 * Mean time of one launch of the current two-step kernel (two lattice
 * steps), as jlb_time_step_kernel.  JLB_E_ARG when two-step kernels are off.
 */
int jlb_time_two_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                             int32_t launches, double *ms_per_launch, void *stream);
/*
 * Multi-step kernels (FP32 / BF16, JLB_MULTI_STEP_VARIANTS of them): one
 * launch takes the state from step n to n + S, S = 3 or 4 (S levels in
 * flight in each wavefront's sweep), bit for bit equal to S single steps.
 * When a variant is selected, jlb_solve runs every graph-captured chunk on
 * it, the averaging window included (there the launch also keeps the
 * contour-stencil fields of its intermediate levels and all S levels are
 * accumulated after it, in time order), and the ramp and the steps before
 * the window's first chunk as pairs of launches, provided the chunk is a
 * multiple of 2 S steps and ny >= rows + S; a four-step variant whose chunk
 * is 4 (mod 8) steps gives way to variant 3 (S3 H10 X4); otherwise the solve
 * runs as without it.  The engine has its own switch (jlb_engine_set_four_step).
 * Variants (depth S, rows per wavefront, halo
 * columns per side: 56 output columns per 64-lane strip with X4, 48 with
 * X8): 0 S4 H10 X4, 1 S4 H12 X4, 2 S4 H16 X4, 3 S3 H10 X4, 4 S3 H12 X4,
 * 5 S4 H12 X8, 6 S3 H7 X4, 7 S3 H8 X4.  jlb_multi_step_shape
 * reports S and the rows of a variant.  Default: 0 (set -1 for none);
 * jlb_autotune selects one when it beats the other kernels per lattice step.
 * jlb_time_multi_step_kernel: mean time of one launch (S lattice steps) of
 * the selected variant, as jlb_time_step_kernel; JLB_E_ARG for FP64, when
 * none is selected or when ny < rows + S.
 */
#define JLB_MULTI_STEP_VARIANTS 8
int jlb_set_multi_step_variant(int32_t precision, int32_t variant);
int jlb_get_multi_step_variant(int32_t precision, int32_t *variant);
int jlb_multi_step_shape(int32_t variant, int32_t *depth, int32_t *rows);
int jlb_time_multi_step_kernel(const jlb_problem *prob, void *workspace, size_t workspace_bytes, int32_t warmup,
                               int32_t launches, double *ms_per_launch, void *stream);
int jlb_get_step_variant(int32_t precision, int32_t *variant);

/*
 * Reference bandwidth: times `launches` runs of a plain device copy of
 * `bytes` bytes (16 bytes per lane, grid-stride) between two device buffers
 * the call allocates, after one warm-up run; *ms_per_launch (host) receives
 * the mean.  Used as the practical peak next to the lattice step and as the
 * known-size kernel that calibrates memory-traffic counters.
 */
int jlb_copy_bandwidth(size_t bytes, int32_t launches, double *ms_per_launch, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched engine: many independent solves resident on one device, stepped  */
/* together by one launch per lattice step over a work list of tiles drawn   */
/* from every admitted solve (Sec. IV design maps are sweeps of independent  */
/* solves).  Requests are admitted while their device footprint fits the    */
/* engine's byte budget; finished solves release their memory, which admits  */
/* waiting requests at the next step boundary (continuous batching).         */
/* ------------------------------------------------------------------------ */

typedef struct jlb_engine jlb_engine;

/* Request status reported by jlb_engine_poll. */
#define JLB_REQ_QUEUED 0
#define JLB_REQ_RUNNING 1
#define JLB_REQ_DONE 2
#define JLB_REQ_FAILED 3
#define JLB_REQ_CANCELLED 4

/*
 * Creates an engine on the current device.
 *   budget_bytes  device bytes the engine may hold for admitted solves
 *   max_slots     most solves resident at once (>= 1)
 *   stream        stream the engine launches on (NULL = a private one)
 * *out receives the handle (host pointer).
 */
int jlb_engine_create(size_t budget_bytes, int32_t max_slots, void *stream, jlb_engine **out);

/* Queues a problem (validated now; JLB_E_ADMISSION if it can never fit the
 * budget); *ticket (host) receives its id.  Never blocks on the device. */
int jlb_engine_submit(jlb_engine *eng, const jlb_problem *prob, uint64_t *ticket);

/* Admits queued requests that fit, then advances every resident solve by up to
 * `steps` lattice steps (rounded up to an even number: the engine works in
 * double steps, one two-step launch for FP32 / BF16 solves when a two-step
 * variant is selected, two single steps otherwise), retiring solves that
 * finish.  *active (host, optional) receives the resident count afterwards. */
int jlb_engine_run(jlb_engine *eng, int64_t steps, int32_t *active);

/* Status of a ticket: *status one of JLB_REQ_*; when DONE, *res holds the
 * outcome (res may be NULL). */
int jlb_engine_poll(jlb_engine *eng, uint64_t ticket, int32_t *status, jlb_result *res);

/* Cancels a queued or resident request and frees its memory. */
int jlb_engine_cancel(jlb_engine *eng, uint64_t ticket);

/* Counts of queued, resident and finished requests and device bytes in use. */
int jlb_engine_stats(jlb_engine *eng, int32_t *queued, int32_t *resident, int32_t *finished, size_t *bytes_in_use);

/*
 * Admission order of queued requests (applied at every chunk boundary, with
 * the byte budget and the slot count as limits):
 *   JLB_POLICY_FIFO  first fit in arrival order (the default);
 *   JLB_POLICY_SJF   smallest work first (cells x steps; ties by arrival) --
 *                    with a slot count below the offered concurrency this
 *                    keeps small requests from waiting behind large ones.
 * max_slots (> 0) replaces the creation-time slot count; 0 keeps it.
 * JLB_E_ARG for an unknown policy or a negative slot count.
 */
#define JLB_POLICY_FIFO 0
#define JLB_POLICY_SJF 1
int jlb_engine_set_policy(jlb_engine *eng, int32_t policy, int32_t max_slots);
/*
 * Four-step rounds (on by default): with `on`, the engine's FP32 / BF16
 * solves that use two-step kernels take one batched four-step launch per
 * round of four steps while four more levels remain (inside the averaging
 * window too), in the shape jlb_engine_four_step_choice reports.  Results
 * are the same bits either way.  Takes effect at the next chunk.  JLB_E_ARG
 * for a null engine.
 */
int jlb_engine_set_four_step(jlb_engine *eng, int32_t on);

/*
 * The engine's four-step shape.  With four-step rounds on, the engine times
 * the batched launch of each four-step variant (0 S4 H10 X4, 1 S4 H12 X4,
 * 2 S4 H16 X4, 5 S4 H12 X8) over the resident solves of a precision that
 * are in four-step mode for the whole next chunk and have ny >= 20, and
 * runs the fastest; it times them again when that set's node count changes
 * by more than a factor of 2.  Before its first timing it runs variant 2.
 * The timing launches change no result.
 *   precision       JLB_FP32 or JLB_BF16
 *   *variant        (host) the multi-step variant the engine runs for that
 *                   precision (-1: no four-step rounds)
 *   ms_per_variant  (host, optional; JLB_MULTI_STEP_VARIANTS entries) the
 *                   last timing's mean ms per batched launch, 0 where not timed
 *   *tunings        (host, optional) timings taken so far, all precisions
 * JLB_E_ARG for a null engine or variant pointer, or FP64.
 */
int jlb_engine_four_step_choice(jlb_engine *eng, int32_t precision, int32_t *variant, double *ms_per_variant,
                                int32_t *tunings);

/* Releases every resource of the engine. */
int jlb_engine_destroy(jlb_engine *eng);

#ifdef __cplusplus
}
#endif

#endif /* JLB_H */
