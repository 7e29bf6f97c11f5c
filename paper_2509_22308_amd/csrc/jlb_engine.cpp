// Batched engine entry points (filled in below the single-solve path).
#include <hip/hip_runtime.h>

#include "../../include/jlb.h"
#include "jlb_host_internal.h"

using namespace jlb;

extern "C" {

int jlb_engine_create(size_t, int32_t, void *, jlb_engine **) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_submit(jlb_engine *, const jlb_problem *, uint64_t *) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_run(jlb_engine *, int64_t, int32_t *) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_poll(jlb_engine *, uint64_t, int32_t *, jlb_result *) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_cancel(jlb_engine *, uint64_t) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_stats(jlb_engine *, int32_t *, int32_t *, int32_t *, size_t *) { return fail(JLB_E_STATE, "engine not built yet"); }
int jlb_engine_destroy(jlb_engine *) { return fail(JLB_E_STATE, "engine not built yet"); }

}
