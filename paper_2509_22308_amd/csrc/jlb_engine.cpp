// Batched engine: many independent solves (the points of a design map, or
// requests as they arrive) resident on one device and stepped together.
//
// Each admitted solve owns a device workspace with the same layout as a
// single solve plus its table of incident-wave values.  Its descriptor in
// device memory carries its step counter and the index of the buffer that
// holds its current state, which the device advances, so a chunk of K
// lattice steps is captured once in a hipGraph and replayed while the set of
// resident solves is unchanged.  The chunk is K / 4 rounds of four steps:
// one batched four-step launch over the (strip, row segment) items of the
// FP32 / BF16 solves with at least four levels to go (its shape timed on
// the resident mix), then the batched
// contour launch of the averaged levels among them (the launch keeps its
// intermediate levels' contour fields when one is averaged), two double steps
// for the others, and the four-step solves' advance-by-four launch.  In a
// double step, solves on single steps (two-step kernels off for their
// precision) take two rounds of one launch per precision over their tiles,
// one batched contour launch and one advance launch, and the others take
// one batched two-step launch per precision over their items (FP64: writing
// both levels' field planes when either is averaged), one two-level contour
// launch and one advance-by-two launch.  Each kernel skips
// the solves that are not its own at their current step.  Solves that finish inside a chunk idle
// (their tiles return at once) until the chunk boundary, where the engine
// reduces their contour sums, returns their memory and admits waiting
// requests that fit the byte budget (continuous batching).
//
// Every per-node operation is the same device code as in a single solve and
// the per-solve sums run in the same order, so a solve's result does not
// depend on what else is resident: it equals the jlb_solve result bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "../../include/jlb.h"
#include "jlb_host_internal.h"

using namespace jlb;

namespace {

constexpr int64_t CHUNK = 128;  // lattice steps per captured graph

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    jlb_problem prob;
    Plan plan;
    int status = JLB_REQ_QUEUED;
    jlb_result res{};
    char *ws = nullptr;       // device: workspace followed by the incident table
    size_t footprint = 0;
    int64_t n = 0;            // host mirror of the device step counter
    int cur = 0;              // host mirror of the device buffer index
    int64_t ramp_end = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double loop_ms_acc = 0;
    // host data of the uploads, prepared ahead while the device runs and
    // released once the admission's copies are done
    std::vector<uint8_t> img;
    std::vector<double> tab;
    bool prepared = false;
};

}  // namespace

struct jlb_engine {
    size_t budget = 0;
    int max_slots = 1;
    int slots_cap = 1;          // slots the device descriptors were sized for
    int policy = JLB_POLICY_FIFO;
    hipStream_t s = nullptr;
    bool own = false;
    uint64_t next_ticket = 1;
    std::map<uint64_t, Request> reqs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> resident;
    size_t in_use = 0;
    int finished = 0;
    // device-side batch description
    SolveDesc *d_desc = nullptr;
    Tile *d_tiles = nullptr;
    size_t tiles_cap = 0;
    int ntiles[3] = {0, 0, 0};
    int tile_off[3] = {0, 0, 0};
    int variant[3] = {0, 0, 0};
    int two[3] = {-1, -1, -1};  // two-step variant per precision (-1: single steps)
    int nitems[3] = {0, 0, 0};  // two-step work items per precision
    int item_off[3] = {0, 0, 0};
    int multi[3] = {-1, -1, -1};  // four-step variant per precision (-1: none)
    int nmitems[3] = {0, 0, 0};   // four-step work items per precision
    int mitem_off[3] = {0, 0, 0};
    bool any_single = false, any_two = false, any_multi = false;
    // per resident solve (in resident order), the launches the captured
    // chunk holds items for: 1 two-step, 2 four-step, 3 both
    std::vector<uint8_t> part;
    bool four_step = true;  // four-step rounds for two-step solves
    // the four-step shape per precision, chosen by timing the batched launch
    // on the resident mix (-1: not timed yet), the times of the last timing
    // and the four-step nodes it was taken on
    int mchoice[3] = {-1, -1, -1};
    double mtune_ms[3][MULTI_STEP_VARIANTS] = {};
    double mtune_nodes[3] = {0.0, 0.0, 0.0};
    int ntunes = 0;
    int max_nc = 0;
    int remap = 0;
    bool dirty = true;
    hipGraphExec_t graph = nullptr;
    double *h_out = nullptr;    // pinned host staging of finished solves' results
    size_t h_out_cap = 0;       // solves it holds
};

namespace {

// The engine steps in rounds of four.  Which four-step shape is fastest
// depends on the resident mix (a few small solves are latency-bound, many
// large ones bound by the halo work per update), so the engine times the
// candidates on the mix itself (tune_four_step); until then it takes the
// one with the least halo work (16-row segments, 4 halo columns).
constexpr int FOUR_STEP_CANDIDATES[] = {MULTI_S4_H10_X4, MULTI_S4_H12_X4, MULTI_S4_H16_X4, MULTI_S4_H12_X8};
constexpr int FOUR_STEP_MAX_ROWS = 16;  // the tallest candidate's segment

int engine_multi_variant(const jlb_engine *e, int p)
{
    if (!e->four_step) return -1;
    return e->mchoice[p] >= 0 ? e->mchoice[p] : MULTI_S4_H16_X4;
}

// Which batched launches a resident solve needs over the next chunk of
// CHUNK steps from its step n: four-step launches while four more levels
// remain (mode checked per round on the device), two-step launches for the
// last one to three steps.  Solves that stay in one mode for the whole chunk get
// items in one list only, so a launch does not spend wavefronts on solves
// that skip it.
uint8_t launch_part(const jlb_engine *e, const Request &r)
{
    const int p = r.plan.prob.precision;
    if (e->two[p] < 0) return 0;
    int depth = 0, rows = 0;
    if (e->multi[p] >= 0) multi_step_shape(e->multi[p], depth, rows);
    if (e->multi[p] < 0 || r.plan.ny < rows + depth) return 1;
    const int64_t total = r.plan.prob.steps;
    if (r.n + depth > total) return 1;           // never in four-step mode again
    if (r.n + CHUNK <= total) return 2;          // four-step mode in every round of the chunk
    return 3;
}

size_t footprint_of(const Plan &q)
{
    const int64_t ramp_end = (int64_t)std::ceil(q.ramp_steps);
    return q.ws_bytes + (size_t)(ramp_end + q.T) * sizeof(double);
}

// Host data of one request's uploads: the mask / contour image and the
// incident values (the ramp steps one by one, then one period indexed by n mod T).
void prepare(Request &r)
{
    if (r.prepared) return;
    const Plan &q = r.plan;
    prepare_upload(q, r.img);
    r.ramp_end = (int64_t)std::ceil(q.ramp_steps);
    r.tab.assign((size_t)(r.ramp_end + q.T), 0.0);
    for (int64_t n = 0; n < r.ramp_end; ++n) r.tab[n] = incident(q, n);
    for (int64_t k = 0; k < q.T; ++k) {
        const int64_t n = r.ramp_end + ((k - r.ramp_end % q.T) + q.T) % q.T;  // first n >= ramp_end with n % T == k
        r.tab[r.ramp_end + k] = incident(q, n);
    }
    r.prepared = true;
}

// Queues the allocation and uploads of one admission; the host data stays
// in the request until the caller has synchronised the stream.
int admit_one(jlb_engine *e, uint64_t t)
{
    Request &r = e->reqs[t];
    const Plan &q = r.plan;
    prepare(r);
    hipError_t err = hipMallocAsync((void **)&r.ws, r.footprint, e->s);
    if (err != hipSuccess) return fail(JLB_E_OOM, "hipMallocAsync(%zu): %s", r.footprint, hipGetErrorString(err));
    int rc = enqueue_upload(q, r.ws, e->s, r.img);
    if (rc) return rc;
    err = hipMemcpyAsync(r.ws + q.ws_bytes, r.tab.data(), r.tab.size() * sizeof(double), hipMemcpyHostToDevice, e->s);
    if (err != hipSuccess) return fail(JLB_E_DEVICE, "engine upload: %s", hipGetErrorString(err));
    r.status = JLB_REQ_RUNNING;
    r.n = 0;
    r.cur = 0;
    r.t_admit = now_ms();
    e->in_use += r.footprint;
    e->resident.push_back(t);
    e->dirty = true;
    return JLB_OK;
}

double work_of(const Request &r) { return (double)r.plan.nx * r.plan.ny * (double)r.plan.prob.steps; }

// Queued requests in the order admission considers them: arrival order, or
// smallest work first.
std::vector<uint64_t> admission_order(jlb_engine *e)
{
    std::vector<uint64_t> order(e->queue.begin(), e->queue.end());
    if (e->policy == JLB_POLICY_SJF)
        std::stable_sort(order.begin(), order.end(),
                         [&](uint64_t a, uint64_t b) { return work_of(e->reqs[a]) < work_of(e->reqs[b]); });
    return order;
}

// Host preparation of the next admissions while the device runs a chunk:
// at most PREPARE_PER_CHUNK requests per call and PREPARE_BYTES of images
// held ahead.
constexpr int PREPARE_PER_CHUNK = 64;
constexpr size_t PREPARE_BYTES = (size_t)256 << 20;
void prepare_ahead(jlb_engine *e)
{
    size_t held = 0;
    int made = 0;
    for (uint64_t t : admission_order(e)) {
        Request &r = e->reqs[t];
        if (!r.prepared) {
            if (made == PREPARE_PER_CHUNK || held + r.plan.ws_bytes > PREPARE_BYTES) break;
            prepare(r);
            ++made;
        }
        held += r.img.size() + r.tab.size() * sizeof(double);
        if (held > PREPARE_BYTES) break;
    }
}

// Admit every queued request that fits, in the policy's order (first fit).
int admit(jlb_engine *e)
{
    const std::vector<uint64_t> order = admission_order(e);
    // every admission of this call is queued first, then one synchronisation
    // covers all their uploads
    int rc = JLB_OK;
    std::vector<uint64_t> taken;
    for (uint64_t t : order) {
        if ((int)e->resident.size() >= e->max_slots) break;
        Request &r = e->reqs[t];
        if (e->in_use + r.footprint > e->budget) continue;
        taken.push_back(t);
        rc = admit_one(e, t);
        if (rc) {
            Request &rr = e->reqs[t];
            rr.status = JLB_REQ_FAILED;
            if (rr.ws) (void)hipFreeAsync(rr.ws, e->s);
            rr.ws = nullptr;
            break;
        }
    }
    if (!taken.empty()) {
        std::sort(taken.begin(), taken.end());
        e->queue.erase(std::remove_if(e->queue.begin(), e->queue.end(),
                                      [&](uint64_t t) { return std::binary_search(taken.begin(), taken.end(), t); }),
                       e->queue.end());
        hipError_t err = hipStreamSynchronize(e->s);
        if (err != hipSuccess && rc == JLB_OK) rc = fail(JLB_E_DEVICE, "engine upload: %s", hipGetErrorString(err));
        for (uint64_t t : taken) {
            Request &r = e->reqs[t];
            std::vector<uint8_t>().swap(r.img);
            std::vector<double>().swap(r.tab);
        }
    }
    return rc;
}

int rebuild(jlb_engine *e)
{
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    const int ns = (int)e->resident.size();
    std::vector<SolveDesc> desc(ns);
    std::vector<Tile> tiles[3], items[3], mitems[3];
    e->max_nc = 0;
    // the resident states together decide whether they stay cache-resident
    size_t working_set = 0;
    for (int k = 0; k < ns; ++k) working_set += 2 * e->reqs[e->resident[k]].plan.state_bytes;
    const int stream_stores = working_set > CACHE_RESIDENT_BYTES ? 1 : 0;
    e->remap = stream_stores ? 0 : 1;
    for (int p = 0; p < 3; ++p) {
        e->variant[p] = jlb::step_variant(p);
        e->two[p] = jlb::two_step_variant(p);
        e->multi[p] = p != JLB_FP64 && e->two[p] >= 0 ? engine_multi_variant(e, p) : -1;
    }
    e->any_single = e->any_two = e->any_multi = false;
    e->part.assign(ns, 0);
    for (int k = 0; k < ns; ++k) {
        Request &r = e->reqs[e->resident[k]];
        const Plan &q = r.plan;
        SolveDesc &d = desc[k];
        memset(&d, 0, sizeof(d));
        d.L = lattice_of(q, (const uint8_t *)(r.ws + q.off_mask));
        d.L.stream_stores = stream_stores;
        d.state[0] = r.ws + q.off_state[0];
        d.state[1] = r.ws + q.off_state[1];
        d.cur = r.cur;
        d.fields = q.prob.precision == JLB_FP64 ? (double *)(r.ws + q.off_fields) : nullptr;
        d.fields_level = (size_t)3 * q.plane;
        d.mid = q.prob.precision == JLB_FP64 ? nullptr : (float *)(r.ws + q.off_mid);
        d.src_tab = (const double *)(r.ws + q.ws_bytes);
        d.ramp_end = r.ramp_end;
        d.T = q.T;
        d.n = r.n;
        d.steps = q.prob.steps;
        d.window = q.window;
        d.C = contour_of(q, r.ws);
        d.precision = q.prob.precision;
        e->max_nc = std::max(e->max_nc, q.nc);
        const int p = q.prob.precision;
        d.two = e->two[p] >= 0 ? 1 : 0;
        if (d.two) {
            const uint8_t part = launch_part(e, r);
            e->part[k] = part;
            // one wavefront per (strip, row segment), in the order the
            // single-solve launch uses for this residency
            int nsx, nsy;
            if (p == JLB_FP64) two_step_shape_f64(e->two[p], q.nx, q.ny, nsx, nsy);
            else two_step_shape(e->two[p], q.nx, q.ny, nsx, nsy);
            if (part & 1) {
                e->any_two = true;
                if (stream_stores) {
                    for (int y = 0; y < nsy; ++y)
                        for (int x = 0; x < nsx; ++x) items[p].push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                } else {
                    for (int x = 0; x < nsx; ++x)
                        for (int y = 0; y < nsy; ++y) items[p].push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                }
            }
            int depth = 0, rows = 0;
            if (e->multi[p] >= 0) multi_step_shape(e->multi[p], depth, rows);
            if (e->multi[p] >= 0 && q.ny >= rows + depth) d.mdepth = depth;
            if (part & 2) {
                // the same orders for the four-step items
                e->any_multi = true;
                int mx, my;
                multi_step_grid(e->multi[p], q.nx, q.ny, mx, my);
                if (stream_stores) {
                    for (int y = 0; y < my; ++y)
                        for (int x = 0; x < mx; ++x) mitems[p].push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                } else {
                    for (int x = 0; x < mx; ++x)
                        for (int y = 0; y < my; ++y) mitems[p].push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                }
            }
            continue;
        }
        e->any_single = true;
        int cols, rows;
        tile_shape(p, e->variant[p], cols, rows);
        const int tx = (q.nx + cols - 1) / cols;
        // tiles cover rows 0..ny (the companion row included)
        const int ty = (q.ny + 1 + rows - 1) / rows;
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) tiles[p].push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
    }
    size_t total = 0;
    for (int p = 0; p < 3; ++p) {
        e->tile_off[p] = (int)total;
        e->ntiles[p] = (int)tiles[p].size();
        total += tiles[p].size();
    }
    for (int p = 0; p < 3; ++p) {
        e->item_off[p] = (int)total;
        e->nitems[p] = (int)items[p].size();
        total += items[p].size();
    }
    for (int p = 0; p < 3; ++p) {
        e->mitem_off[p] = (int)total;
        e->nmitems[p] = (int)mitems[p].size();
        total += mitems[p].size();
    }
    hipError_t err = hipSuccess;
    if (!e->d_desc) {
        e->slots_cap = e->max_slots;
        err = hipMallocAsync((void **)&e->d_desc, sizeof(SolveDesc) * e->slots_cap, e->s);
    }
    if (err == hipSuccess && total > e->tiles_cap) {
        if (e->d_tiles) (void)hipFreeAsync(e->d_tiles, e->s);
        e->tiles_cap = std::max(total, 2 * e->tiles_cap);
        err = hipMallocAsync((void **)&e->d_tiles, sizeof(Tile) * e->tiles_cap, e->s);
    }
    if (err == hipSuccess && ns > 0)
        err = hipMemcpyAsync(e->d_desc, desc.data(), sizeof(SolveDesc) * ns, hipMemcpyHostToDevice, e->s);
    for (int p = 0; p < 3 && err == hipSuccess; ++p) {
        if (!tiles[p].empty())
            err = hipMemcpyAsync(e->d_tiles + e->tile_off[p], tiles[p].data(), sizeof(Tile) * tiles[p].size(),
                                 hipMemcpyHostToDevice, e->s);
        if (err == hipSuccess && !items[p].empty())
            err = hipMemcpyAsync(e->d_tiles + e->item_off[p], items[p].data(), sizeof(Tile) * items[p].size(),
                                 hipMemcpyHostToDevice, e->s);
        if (err == hipSuccess && !mitems[p].empty())
            err = hipMemcpyAsync(e->d_tiles + e->mitem_off[p], mitems[p].data(), sizeof(Tile) * mitems[p].size(),
                                 hipMemcpyHostToDevice, e->s);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(e->s);  // host vectors go out of scope
    if (err != hipSuccess) return fail(JLB_E_DEVICE, "engine rebuild: %s", hipGetErrorString(err));
    e->dirty = false;
    return JLB_OK;
}

// One double step: two single steps of the single-step solves, one two-step
// launch of the others.
hipError_t launch_double_step(jlb_engine *e)
{
    const int ns = (int)e->resident.size();
    hipError_t err = hipSuccess;
    for (int r = 0; r < 2 && e->any_single && err == hipSuccess; ++r) {
        for (int p = 0; p < 3 && err == hipSuccess; ++p)
            err = launch_step_batch(p, e->variant[p], e->d_desc, e->d_tiles + e->tile_off[p], e->ntiles[p], e->remap,
                                    e->s);
        if (err == hipSuccess) err = launch_contour_batch(e->d_desc, ns, e->max_nc, e->s);
        if (err == hipSuccess) err = launch_advance(e->d_desc, ns, 0, e->s);
    }
    if (e->any_two && err == hipSuccess) {
        for (int p = 0; p < 3 && err == hipSuccess; ++p)
            if (e->nitems[p] > 0)
                err = p == JLB_FP64 ? launch_step2_f64_batch(e->two[p], e->d_desc, e->d_tiles + e->item_off[p],
                                                             e->nitems[p], e->remap, e->s)
                                    : launch_step2_batch(p, e->two[p], e->d_desc, e->d_tiles + e->item_off[p],
                                                         e->nitems[p], e->remap, e->s);
        if (err == hipSuccess) err = launch_contour2_batch(e->d_desc, ns, e->max_nc, e->s);
        if (err == hipSuccess) err = launch_advance(e->d_desc, ns, 1, e->s);
    }
    return err;
}

// Four steps: one four-step launch of the solves in multi mode, two double
// steps of the others, then the four-step solves' advance.
hipError_t launch_quad_step(jlb_engine *e)
{
    const int ns = (int)e->resident.size();
    hipError_t err = hipSuccess;
    for (int p = 1; p < 3 && e->any_multi && err == hipSuccess; ++p)
        if (e->nmitems[p] > 0)
            err = launch_stepm_batch(p, e->multi[p], e->d_desc, e->d_tiles + e->mitem_off[p], e->nmitems[p], e->remap,
                                     e->s);
    if (e->any_multi && err == hipSuccess) err = launch_contourm_batch(e->d_desc, ns, e->max_nc, e->s);
    for (int k = 0; k < 2 && err == hipSuccess; ++k) err = launch_double_step(e);
    if (e->any_multi && err == hipSuccess) err = launch_advance(e->d_desc, ns, 2, e->s);
    return err;
}

// Times the batched four-step launch of every candidate shape over the
// solves of each FP32 / BF16 precision that are in four-step mode for the
// whole next chunk (those every candidate can take: ny >= 20), when that
// set's node count differs by more than a factor of 2 from the one of the
// last timing, and keeps the fastest.  The timed launches write only what
// the next real launch writes again before anything reads it (the other
// state buffer, the window's intermediate contour fields); no solve's step
// counter moves.  *changed: a precision's shape changed (the caller
// rebuilds).
int tune_four_step(jlb_engine *e, bool &changed)
{
    changed = false;
    if (!e->four_step || !e->any_multi) return JLB_OK;
    const bool row_major = e->remap == 0;  // the order rebuild() uses for this residency
    for (int p = 1; p < 3; ++p) {
        if (e->multi[p] < 0) continue;
        std::vector<int> ks;
        double nodes = 0.0;
        for (size_t k = 0; k < e->resident.size(); ++k) {
            const Plan &q = e->reqs[e->resident[k]].plan;
            if (q.prob.precision != p || !(e->part[k] & 2) || q.ny < FOUR_STEP_MAX_ROWS + 4) continue;
            ks.push_back((int)k);
            nodes += (double)q.nx * q.ny;
        }
        if (ks.empty()) continue;
        const double last = e->mtune_nodes[p];
        if (last > 0.0 && nodes <= 2.0 * last && 2.0 * nodes >= last) continue;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        hipError_t err = hipEventCreate(&ev0);
        if (err == hipSuccess) err = hipEventCreate(&ev1);
        double ms_of[MULTI_STEP_VARIANTS] = {};
        int best = -1;
        for (int v : FOUR_STEP_CANDIDATES) {
            if (err != hipSuccess) break;
            std::vector<Tile> items;
            for (int k : ks) {
                const Plan &q = e->reqs[e->resident[k]].plan;
                int mx, my;
                multi_step_grid(v, q.nx, q.ny, mx, my);
                if (row_major) {
                    for (int y = 0; y < my; ++y)
                        for (int x = 0; x < mx; ++x) items.push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                } else {
                    for (int x = 0; x < mx; ++x)
                        for (int y = 0; y < my; ++y) items.push_back(Tile{(uint32_t)k, (uint16_t)x, (uint16_t)y});
                }
            }
            Tile *d_items = nullptr;
            err = hipMallocAsync((void **)&d_items, sizeof(Tile) * items.size(), e->s);
            if (err == hipSuccess)
                err = hipMemcpyAsync(d_items, items.data(), sizeof(Tile) * items.size(), hipMemcpyHostToDevice, e->s);
            const int n = (int)items.size();
            if (err == hipSuccess) err = launch_stepm_batch(p, v, e->d_desc, d_items, n, e->remap, e->s);  // warm-up
            if (err == hipSuccess) err = hipEventRecord(ev0, e->s);
            constexpr int TIMED = 3;
            for (int i = 0; i < TIMED && err == hipSuccess; ++i)
                err = launch_stepm_batch(p, v, e->d_desc, d_items, n, e->remap, e->s);
            if (err == hipSuccess) err = hipEventRecord(ev1, e->s);
            if (err == hipSuccess) err = hipEventSynchronize(ev1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev0, ev1);
            if (d_items) (void)hipFreeAsync(d_items, e->s);
            if (err != hipSuccess) break;
            ms_of[v] = ms / TIMED;
            if (best < 0 || ms_of[v] < ms_of[best]) best = v;
        }
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (err == hipSuccess) err = hipStreamSynchronize(e->s);
        if (err != hipSuccess) return fail(JLB_E_DEVICE, "engine four-step timing: %s", hipGetErrorString(err));
        std::copy(ms_of, ms_of + MULTI_STEP_VARIANTS, e->mtune_ms[p]);
        e->mtune_nodes[p] = nodes;
        e->ntunes += 1;
        if (best != e->multi[p]) changed = true;
        e->mchoice[p] = best;
    }
    return JLB_OK;
}

int capture(jlb_engine *e)
{
    hipGraph_t g;
    if (hipStreamBeginCapture(e->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(JLB_E_DEVICE, "engine capture begin");
    hipError_t err = hipSuccess;
    for (int64_t k = 0; k < CHUNK / 4 && err == hipSuccess; ++k) err = launch_quad_step(e);
    hipError_t err2 = hipStreamEndCapture(e->s, &g);
    if (err != hipSuccess || err2 != hipSuccess) return fail(JLB_E_DEVICE, "engine capture failed");
    err = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return fail(JLB_E_DEVICE, "engine graph instantiate: %s", hipGetErrorString(err));
    return JLB_OK;
}

// Reduces and returns every resident solve whose steps are all done.
int harvest(jlb_engine *e)
{
    // finished solves: reduce each, copy every result to pinned host memory,
    // then one synchronisation
    std::vector<size_t> done;
    for (size_t k = 0; k < e->resident.size(); ++k)
        if (e->reqs[e->resident[k]].n >= e->reqs[e->resident[k]].plan.prob.steps) done.push_back(k);
    if (done.empty()) return JLB_OK;
    if (e->h_out_cap < done.size()) {
        if (e->h_out) (void)hipHostFree(e->h_out);
        e->h_out = nullptr;
        e->h_out_cap = 0;
        const size_t cap = std::max<size_t>(done.size(), (size_t)e->max_slots);
        if (hipHostMalloc((void **)&e->h_out, cap * 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(JLB_E_OOM, "pinned result staging");
        e->h_out_cap = cap;
    }
    hipError_t err = hipSuccess;
    for (size_t d = 0; d < done.size() && err == hipSuccess; ++d) {
        Request &r = e->reqs[e->resident[done[d]]];
        const Plan &q = r.plan;
        const ContourDev C = contour_of(q, r.ws);
        const double f0 = M_PI * q.prob.radius * q.prob.e0 * q.prob.e0 / 4.0;
        err = launch_reduce(C, 1.0 / (double)q.window, f0, 2.0 * f0 * q.prob.radius, (double *)(r.ws + q.off_out), e->s);
        if (err == hipSuccess) {
            // the final fields: FP64 keeps them in the field planes of the last level's parity
            // (written through the window), the others in the state buffer that holds the last level
            const Lattice L = lattice_of(q, (const uint8_t *)(r.ws + q.off_mask));
            const void *fld = q.prob.precision == JLB_FP64
                                  ? (const void *)(r.ws + q.off_fields + (size_t)(q.prob.steps & 1) * 3 * q.plane * sizeof(double))
                                  : r.ws + q.off_state[r.cur];
            err = launch_energy(q.prob.precision, L, fld, (double *)(r.ws + q.off_parts), q.nparts,
                                (double *)(r.ws + q.off_out) + 6, e->s);
        }
        if (err == hipSuccess)
            err = hipMemcpyAsync(e->h_out + 8 * d, r.ws + q.off_out, 7 * sizeof(double), hipMemcpyDeviceToHost, e->s);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(e->s);
    if (err != hipSuccess) return fail(JLB_E_DEVICE, "engine harvest: %s", hipGetErrorString(err));
    const double t_done = now_ms();
    for (size_t d = 0; d < done.size(); ++d) {
        Request &r = e->reqs[e->resident[done[d]]];
        const Plan &q = r.plan;
        const double *out = e->h_out + 8 * d;
        r.res.fx = out[0];
        r.res.fy = out[1];
        r.res.tz = out[2];
        r.res.fx_raw = out[3];
        r.res.fy_raw = out[4];
        r.res.tz_raw = out[5];
        r.res.steps_done = q.prob.steps;
        r.res.window_steps = q.window;
        r.res.contour_points = q.nc;
        r.res.graph_used = 1;
        r.res.bytes_per_step = (int64_t)q.bytes_per_lup * q.nx * q.ny;
        r.res.state_passes = q.prob.steps;
        r.res.energy_final = out[6];
        r.t_done = t_done;
        r.res.total_ms = r.t_done - r.t_submit;
        r.res.loop_ms = r.t_done - r.t_admit;
        bool finite = true;
        for (int i = 0; i < 6; ++i) finite = finite && std::isfinite(out[i]);
        r.status = finite ? JLB_REQ_DONE : JLB_REQ_FAILED;
        (void)hipFreeAsync(r.ws, e->s);
        r.ws = nullptr;
        e->in_use -= r.footprint;
        e->finished += 1;
    }
    // drop the finished ones from the resident list, keeping the others' order
    std::vector<uint64_t> keep;
    keep.reserve(e->resident.size() - done.size());
    for (size_t k = 0, d = 0; k < e->resident.size(); ++k) {
        if (d < done.size() && done[d] == k) { ++d; continue; }
        keep.push_back(e->resident[k]);
    }
    e->resident.swap(keep);
    e->dirty = true;
    return JLB_OK;
}

}  // namespace

extern "C" {

int jlb_engine_create(size_t budget_bytes, int32_t max_slots, void *stream, jlb_engine **out)
{
    clear_error();
    if (!out || max_slots < 1 || budget_bytes == 0) return fail(JLB_E_ARG, "bad engine arguments");
    jlb_engine *e = new jlb_engine();
    e->budget = budget_bytes;
    e->max_slots = max_slots;
    e->slots_cap = max_slots;
    if (stream) {
        e->s = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) != hipSuccess) {
            delete e;
            return fail(JLB_E_DEVICE, "cannot create the engine stream");
        }
        e->own = true;
    }
    *out = e;
    return JLB_OK;
}

int jlb_engine_submit(jlb_engine *e, const jlb_problem *prob, uint64_t *ticket)
{
    clear_error();
    if (!e || !prob || !ticket) return fail(JLB_E_ARG, "null argument");
    if (prob->plateau_tol != 0.0) return fail(JLB_E_ARG, "the plateau stop is a single-solve option");
    Request r;
    r.prob = *prob;
    int rc = make_plan(prob, &r.plan);
    if (rc) return rc;
    r.footprint = footprint_of(r.plan);
    if (r.footprint > e->budget)
        return fail(JLB_E_ADMISSION, "request needs %zu bytes, budget is %zu", r.footprint, e->budget);
    r.t_submit = now_ms();
    const uint64_t t = e->next_ticket++;
    e->reqs.emplace(t, r);
    e->queue.push_back(t);
    *ticket = t;
    return JLB_OK;
}

int jlb_engine_run(jlb_engine *e, int64_t steps, int32_t *active)
{
    clear_error();
    if (!e || steps < 0) return fail(JLB_E_ARG, "bad arguments");
    int rc = admit(e);
    if (rc) return rc;
    int64_t done = 0;
    while (done < steps && !e->resident.empty()) {
        if (e->dirty) {
            rc = rebuild(e);
            if (rc) return rc;
        }
        // a solve that changed launch part since the capture needs new item lists
        for (size_t j = 0; j < e->resident.size() && !e->dirty; ++j)
            if (launch_part(e, e->reqs[e->resident[j]]) != e->part[j]) e->dirty = true;
        if (e->dirty) {
            rc = rebuild(e);
            if (rc) return rc;
        }
        // the four-step shape for this mix
        bool retuned = false;
        rc = tune_four_step(e, retuned);
        if (rc) return rc;
        if (retuned) {
            rc = rebuild(e);
            if (rc) return rc;
        }
        // whole double steps
        const int64_t k = std::min<int64_t>(CHUNK, (steps - done + 1) / 2 * 2);
        if (k == CHUNK) {
            if (!e->graph) {
                rc = capture(e);
                if (rc) return rc;
            }
            if (hipGraphLaunch(e->graph, e->s) != hipSuccess) return fail(JLB_E_DEVICE, "engine graph launch");
            // host work for the next admissions while the chunk runs
            prepare_ahead(e);
        } else {
            for (int64_t i = 0; i < k / 4; ++i)
                if (launch_quad_step(e) != hipSuccess) return fail(JLB_E_DEVICE, "engine step launch");
            if (k % 4 && launch_double_step(e) != hipSuccess) return fail(JLB_E_DEVICE, "engine step launch");
        }
        // host mirrors of the device counters (the advance kernels' rules)
        for (uint64_t t : e->resident) {
            Request &r = e->reqs[t];
            const int64_t total = r.plan.prob.steps;
            const int p = r.plan.prob.precision;
            const bool two = e->two[p] >= 0;
            int mdepth = 0, mrows = 0;
            if (two && e->multi[p] >= 0) multi_step_shape(e->multi[p], mdepth, mrows);
            if (r.plan.ny < mrows + mdepth) mdepth = 0;
            auto multi_mode = [&] { return mdepth > 0 && r.n + mdepth <= total; };
            auto double_step = [&] {
                for (int i = 0; i < (two ? 1 : 2) && r.n < total; ++i) {
                    if (two && multi_mode()) return;
                    r.n = two ? std::min<int64_t>(r.n + 2, total) : r.n + 1;
                    r.cur ^= 1;
                }
            };
            for (int64_t i = 0; i < k / 4; ++i) {
                if (r.n < total && multi_mode()) {
                    r.n += mdepth;
                    r.cur ^= 1;
                } else {
                    double_step();
                    double_step();
                }
            }
            if (k % 4) double_step();
        }
        done += k;
        rc = harvest(e);
        if (rc) return rc;
        rc = admit(e);
        if (rc) return rc;
    }
    if (hipStreamSynchronize(e->s) != hipSuccess) return fail(JLB_E_DEVICE, "engine sync");
    if (active) *active = (int32_t)e->resident.size();
    return JLB_OK;
}

int jlb_engine_poll(jlb_engine *e, uint64_t ticket, int32_t *status, jlb_result *res)
{
    clear_error();
    if (!e || !status) return fail(JLB_E_ARG, "null argument");
    auto it = e->reqs.find(ticket);
    if (it == e->reqs.end()) return fail(JLB_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    *status = it->second.status;
    if (res) *res = it->second.res;
    return JLB_OK;
}

int jlb_engine_cancel(jlb_engine *e, uint64_t ticket)
{
    clear_error();
    if (!e) return fail(JLB_E_ARG, "null engine");
    auto it = e->reqs.find(ticket);
    if (it == e->reqs.end()) return fail(JLB_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    Request &r = it->second;
    if (r.status == JLB_REQ_QUEUED) {
        e->queue.erase(std::remove(e->queue.begin(), e->queue.end(), ticket), e->queue.end());
        std::vector<uint8_t>().swap(r.img);  // host data prepared ahead
        std::vector<double>().swap(r.tab);
        r.prepared = false;
    } else if (r.status == JLB_REQ_RUNNING) {
        if (hipStreamSynchronize(e->s) != hipSuccess) return fail(JLB_E_DEVICE, "engine sync");
        (void)hipFreeAsync(r.ws, e->s);
        r.ws = nullptr;
        e->in_use -= r.footprint;
        e->resident.erase(std::remove(e->resident.begin(), e->resident.end(), ticket), e->resident.end());
        e->dirty = true;
    } else {
        return fail(JLB_E_STATE, "ticket %llu already finished", (unsigned long long)ticket);
    }
    r.status = JLB_REQ_CANCELLED;
    return JLB_OK;
}

int jlb_engine_set_four_step(jlb_engine *e, int32_t on)
{
    clear_error();
    if (!e) return fail(JLB_E_ARG, "null engine");
    if (e->four_step != (on != 0)) {
        e->four_step = on != 0;
        e->dirty = true;
    }
    return JLB_OK;
}

int jlb_engine_four_step_choice(jlb_engine *e, int32_t precision, int32_t *variant, double *ms_per_variant,
                                int32_t *tunings)
{
    clear_error();
    if (!e || !variant) return fail(JLB_E_ARG, "null argument");
    if (precision != JLB_FP32 && precision != JLB_BF16) return fail(JLB_E_ARG, "four-step rounds are FP32 / BF16");
    *variant = jlb::two_step_variant(precision) >= 0 ? engine_multi_variant(e, precision) : -1;
    if (ms_per_variant) std::copy(e->mtune_ms[precision], e->mtune_ms[precision] + MULTI_STEP_VARIANTS, ms_per_variant);
    if (tunings) *tunings = e->ntunes;
    return JLB_OK;
}

int jlb_engine_set_policy(jlb_engine *e, int32_t policy, int32_t max_slots)
{
    clear_error();
    if (!e) return fail(JLB_E_ARG, "null engine");
    if (policy != JLB_POLICY_FIFO && policy != JLB_POLICY_SJF) return fail(JLB_E_ARG, "unknown policy %d", policy);
    if (max_slots < 0) return fail(JLB_E_ARG, "negative slot count");
    // the device descriptor array, once allocated, bounds the slot count
    if (max_slots > 0 && e->d_desc && max_slots > e->slots_cap)
        return fail(JLB_E_ARG, "slot count %d above the %d the engine was created with", max_slots, e->slots_cap);
    e->policy = policy;
    if (max_slots > 0) e->max_slots = max_slots;
    return JLB_OK;
}

int jlb_engine_stats(jlb_engine *e, int32_t *queued, int32_t *resident, int32_t *finished, size_t *bytes_in_use)
{
    clear_error();
    if (!e) return fail(JLB_E_ARG, "null engine");
    if (queued) *queued = (int32_t)e->queue.size();
    if (resident) *resident = (int32_t)e->resident.size();
    if (finished) *finished = e->finished;
    if (bytes_in_use) *bytes_in_use = e->in_use;
    return JLB_OK;
}

int jlb_engine_destroy(jlb_engine *e)
{
    clear_error();
    if (!e) return fail(JLB_E_ARG, "null engine");
    (void)hipStreamSynchronize(e->s);
    if (e->graph) (void)hipGraphExecDestroy(e->graph);
    for (auto &kv : e->reqs)
        if (kv.second.ws) (void)hipFreeAsync(kv.second.ws, e->s);
    if (e->d_desc) (void)hipFreeAsync(e->d_desc, e->s);
    if (e->d_tiles) (void)hipFreeAsync(e->d_tiles, e->s);
    (void)hipStreamSynchronize(e->s);
    if (e->h_out) (void)hipHostFree(e->h_out);
    if (e->own) (void)hipStreamDestroy(e->s);
    delete e;
    return JLB_OK;
}

}  // extern "C"
