// Plan files are not implemented: these entry points report SPTRSV_ERR_STATE
// with a message and do no work (a plan is rebuilt by sptrsv_analyze and
// sptrsv_rewrite, which take well under a second on the benchmark matrices).
#include "common.h"

#define PENDING(h) return set_err((h), SPTRSV_ERR_STATE, "%s: plan files are not implemented", __func__)

extern "C" {
sptrsv_status_t sptrsv_plan_save(sptrsv_handle_t h, const char *) { PENDING(h); }
sptrsv_status_t sptrsv_plan_load(sptrsv_handle_t h, const char *) { PENDING(h); }
}
