// Entry points whose kernels are not built yet: they validate nothing and
// report TTC_ERR_UNSUPPORTED.
#include <string>
#include "ttc_internal.h"

namespace ttc { ttc_status fail(ttc_status s, const std::string& msg); }
using ttc::fail;

extern "C" {
ttc_status ttm_apply_dense_query(const ttc_ttm*, int64_t, ttc_prec, ttc_sched, int32_t, size_t*) {
  return fail(TTC_ERR_UNSUPPORTED, "not built");
}
ttc_status ttm_apply_dense(const ttc_ttm*, const void*, int64_t, void*, ttc_prec, ttc_sched, void*, size_t, void*) {
  return fail(TTC_ERR_UNSUPPORTED, "not built");
}
ttc_status ttm_apply_dense_bwd(const ttc_ttm*, const void*, const void*, int64_t, void*, void* const*, ttc_prec,
                               ttc_sched, void*, size_t, void*) {
  return fail(TTC_ERR_UNSUPPORTED, "not built");
}
ttc_status ttc_mse_loss_query(int64_t, size_t*) { return fail(TTC_ERR_UNSUPPORTED, "not built"); }
ttc_status ttc_mse_loss(const float*, const float*, int64_t, double*, float*, void*, size_t, void*) {
  return fail(TTC_ERR_UNSUPPORTED, "not built");
}
ttc_status tt_batch_plan_create(const ttc_pair*, int32_t, uint32_t, ttc_prec, ttc_plan**) {
  return fail(TTC_ERR_UNSUPPORTED, "not built");
}
ttc_status tt_batch_plan_info(const ttc_plan*, int64_t*, double*, double*) { return fail(TTC_ERR_UNSUPPORTED, "not built"); }
ttc_status tt_batch_run(ttc_plan*, double*, float*, void*) { return fail(TTC_ERR_UNSUPPORTED, "not built"); }
ttc_status tt_batch_run_plain(ttc_plan*, double*, float*, void*) { return fail(TTC_ERR_UNSUPPORTED, "not built"); }
void tt_batch_plan_destroy(ttc_plan*) {}
}
