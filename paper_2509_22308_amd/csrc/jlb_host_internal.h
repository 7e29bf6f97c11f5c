// Host-side helpers shared by the single-solve driver and the batched engine.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <vector>

#include "../../include/jlb.h"
#include "jlb_internal.h"

namespace jlb {

// Every derived quantity of one solve, including its device workspace layout.
struct Plan {
    jlb_problem prob;
    int nx, ny, pitch;
    size_t plane;           // elements per population plane ((ny + 1) * pitch)
    double period;          // 3 lambda
    int64_t T;              // period in whole steps
    double omega;           // 2 pi / period
    double ramp_steps;      // ramp_periods * period
    int64_t window;         // avg_periods * T
    double cx, cy, rc;      // centre and contour radius
    int nc;                 // contour samples
    double eps[4];          // permittivity per material id
    size_t state_bytes;     // one state buffer
    int bytes_per_lup;      // algorithmic HBM bytes per lattice update
    size_t off_state[2], off_fields, off_mid, off_mask, off_i0, off_j0, off_wx, off_wy, off_nxk, off_nyk, off_acc,
        off_dft, off_out, off_parts;
    int nparts;
    size_t ws_bytes;
};

struct ContourHost {
    std::vector<int> i0, j0;
    std::vector<double> wx, wy, nxk, nyk;
};

int fail(int code, const char *fmt, ...);
void clear_error();
const char *last_error();

int make_plan(const jlb_problem *p, Plan *pl);
void material_map(const Plan &q, uint8_t *mat, size_t row_stride);
void build_mask(const Plan &q, std::vector<uint8_t> &mask);
void build_contour(const Plan &q, ContourHost &c);
double incident(const Plan &q, int64_t n);
hipStream_t own_stream();
// Largest state pair (bytes, both buffers) a single solve of this precision
// keeps cache-resident.
size_t resident_limit(int precision);
Lattice lattice_of(const Plan &q, const uint8_t *dmask);
ContourDev contour_of(const Plan &q, char *ws);
int upload_setup(const Plan &q, char *ws, hipStream_t s);
// upload_setup in two halves: the host image of the mask and contour tables
// (host work only), then its copy and the zeroing of the device state on `s`
// (asynchronous: `img` must stay alive until the stream has passed the copy).
void prepare_upload(const Plan &q, std::vector<uint8_t> &img);
int enqueue_upload(const Plan &q, char *ws, hipStream_t s, const std::vector<uint8_t> &img);
int step_variant(int precision);
// Two-step variant of a precision (-1: single steps only; always -1 for FP64).
int two_step_variant(int precision);
int multi_step_variant(int precision);
// Optional outputs of a solve: the far field at nphi angles into the device
// array s2, and the instantaneous force trace [steps][3] (nullptr: none).
struct FarOut {
    int nphi;
    double *s2;
    double *force = nullptr;
};
int run_solve(const Plan &q, char *ws, jlb_result *res, double *ez, double *hx, double *hy, double *energy,
              hipStream_t s, FarOut far = {0, nullptr}, bool events = true);

}  // namespace jlb
