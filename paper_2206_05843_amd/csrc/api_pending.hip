// Entry points whose kernels are not in this file set yet: they report
// SPTRSV_ERR_STATE with a message instead of doing any work.
#include "common.h"

#define PENDING(h) return set_err((h), SPTRSV_ERR_STATE, "%s: not available in this build", __func__)

extern "C" {
sptrsv_status_t sptrsv_batch_analyze(sptrsv_handle_t h, int32_t, const int32_t *, const int64_t *, const int64_t *,
                                     const int32_t *, const int32_t *, const double *, hipStream_t) {
  PENDING(h);
}
sptrsv_status_t sptrsv_batch_solve(sptrsv_handle_t h, int32_t, const double *, double *, hipStream_t) { PENDING(h); }
sptrsv_status_t sptrsv_batch_solve_looped(sptrsv_handle_t h, int32_t, const double *, double *, hipStream_t) {
  PENDING(h);
}
sptrsv_status_t sptrsv_batch_levels(sptrsv_handle_t h, int32_t, int32_t *, int32_t *, int32_t *, hipStream_t) {
  PENDING(h);
}
sptrsv_status_t sptrsv_plan_save(sptrsv_handle_t h, const char *) { PENDING(h); }
sptrsv_status_t sptrsv_plan_load(sptrsv_handle_t h, const char *) { PENDING(h); }
}
