// Entry points whose work is not in this file set yet: they report
// SPTRSV_ERR_STATE with a message instead of doing any work.
#include "common.h"

#define PENDING(h) return set_err((h), SPTRSV_ERR_STATE, "%s: not available in this build", __func__)

extern "C" {
sptrsv_status_t sptrsv_plan_save(sptrsv_handle_t h, const char *) { PENDING(h); }
sptrsv_status_t sptrsv_plan_load(sptrsv_handle_t h, const char *) { PENDING(h); }
}
