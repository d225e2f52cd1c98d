// Serving loop of libabm (abm_submit / abm_poll / abm_cancel).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "abm_runtime.h"

namespace abm {

void serve_shutdown(abm_ctx* ctx) { (void)ctx; }

}  // namespace abm

using namespace abm;

extern "C" {

abm_status abm_submit(abm_ctx* ctx, const abm_problem* prob, double* y_out, uint64_t* ticket)
{
    (void)ctx;
    (void)prob;
    (void)y_out;
    (void)ticket;
    return fail(ABM_EINVAL, "serving loop not available in this build");
}

abm_status abm_poll(abm_ctx* ctx, uint64_t ticket, abm_result* res)
{
    (void)ctx;
    (void)ticket;
    (void)res;
    return fail(ABM_ENOENT, "serving loop not available in this build");
}

abm_status abm_cancel(abm_ctx* ctx, uint64_t ticket)
{
    (void)ctx;
    (void)ticket;
    return fail(ABM_ENOENT, "serving loop not available in this build");
}

}  // extern "C"
