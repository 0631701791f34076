// placeholder, replaced by the batched persistent evaluation
#include "common.hpp"
extern "C" {
int spline_batch_plan_create(const spl_item*, int32_t, const int32_t*, void*, void**) { return pws::fail(SPL_EUNSUPPORTED, "batched evaluation not built"); }
int spline_batch_eval_vgl(void*, void*) { return pws::fail(SPL_EUNSUPPORTED, "batched evaluation not built"); }
int spline_batch_graph_launch(void*, void*) { return pws::fail(SPL_EUNSUPPORTED, "batched evaluation not built"); }
void spline_batch_plan_destroy(void*) {}
int spline_batch_plan_info(void*, int64_t*, int64_t*) { return pws::fail(SPL_EUNSUPPORTED, "batched evaluation not built"); }
}
