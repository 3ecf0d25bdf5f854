// Schedule selection for the AUTO policy: exhaustive tuner and cost model.
// (Filled in by the tuner / model implementation.)
#include "runtime_internal.h"

struct ModelState {};

void upir_model_free(upir_ctx *c) {
  delete c->model;
  c->model = nullptr;
}

namespace upir {
int candidate_count(upir_ctx *, const upir_loop_obj *) { return 0; }
bool candidate_at(upir_ctx *, const upir_loop_obj *, int, upir_spmd &, upir_sched &) { return false; }
void candidate_features(upir_ctx *, const upir_loop_obj *, const upir_spmd &, const upir_sched &, float f[32]) {
  for (int i = 0; i < 32; ++i) f[i] = 0.0f;
}
bool model_pick(upir_ctx *, upir_loop_obj *, upir_spmd &, upir_sched &) { return false; }
}  // namespace upir

#define NOTYET(c) return upir_fail(c, UPIR_EUNSUPPORTED, "not built yet")

extern "C" {
upir_status upir_tune(upir_ctx *c, const upir_spmd *, upir_loop_h, int32_t, upir_sched *, upir_spmd *, double *) { NOTYET(c); }
upir_status upir_candidates(upir_ctx *c, upir_loop_h, int32_t *) { NOTYET(c); }
upir_status upir_candidate_features(upir_ctx *c, upir_loop_h, int32_t, float *, upir_spmd *, upir_sched *) { NOTYET(c); }
upir_status upir_tune_db_save(upir_ctx *c, const char *) { NOTYET(c); }
upir_status upir_tune_db_load(upir_ctx *c, const char *) { NOTYET(c); }
upir_status upir_tune_db_size(upir_ctx *c, int64_t *) { NOTYET(c); }
upir_status upir_tune_db_row(upir_ctx *c, int64_t, float *, float *, int64_t *) { NOTYET(c); }
upir_status upir_model_init(upir_ctx *c, uint64_t) { NOTYET(c); }
upir_status upir_model_set_params(upir_ctx *c, const float *) { NOTYET(c); }
upir_status upir_model_get_params(upir_ctx *c, float *) { NOTYET(c); }
upir_status upir_model_forward(upir_ctx *c, const float *, int64_t, float *) { NOTYET(c); }
upir_status upir_model_step(upir_ctx *c, const float *, const float *, int64_t, float, int32_t, float *, float *) { NOTYET(c); }
upir_status upir_model_train(upir_ctx *c, int32_t, int32_t, float, int32_t, float *, float *) { NOTYET(c); }
upir_status upir_model_enable(upir_ctx *c, int32_t) { NOTYET(c); }
upir_status upir_model_save(upir_ctx *c, const char *) { NOTYET(c); }
upir_status upir_model_load(upir_ctx *c, const char *) { NOTYET(c); }
}
