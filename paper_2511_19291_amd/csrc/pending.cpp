// pending.cpp -- entry points whose kernels are not built yet.
#include "sv_internal.h"

extern "C" {
static sv_status pending(const char* what)
{
    (void)what;
    return SV_ERR_UNSUPPORTED;
}
sv_status sv_batch_plan_create(int, const int*, const sv_op* const*, const int*, const int*, void*, sv_batch_plan*) { return pending("batch"); }
sv_status sv_batch_param_layout(sv_batch_plan, int64_t*, int64_t*) { return pending("batch"); }
sv_status sv_batch_launch(sv_batch_plan, const double*, double*) { return pending("batch"); }
sv_status sv_batch_launch_pergate(sv_batch_plan, const double*, double*) { return pending("batch"); }
sv_status sv_batch_plan_free(sv_batch_plan) { return pending("batch"); }
}
