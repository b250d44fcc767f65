// fno_host.cpp -- network entry points (placeholder until the network
// kernels are linked in).
#include <hip/hip_runtime.h>

#include "../../include/mdpnop.h"
#include "host_internal.h"

using namespace mdp;

void mdp::Ctx::release_fno() {}

extern "C" tr_status no_model_create(tr_context* ctx, no_model** m, int32_t,
                                     int32_t, int32_t, int32_t, const float*) {
    if (m) *m = nullptr;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (c) c->fail("network kernels not built");
    return TR_ERR_INVALID_ARG;
}
extern "C" void no_model_destroy(no_model*) {}
extern "C" int64_t no_model_param_count(const no_model*) { return 0; }
extern "C" tr_status no_model_get_params(tr_context*, const no_model*, float*) {
    return TR_ERR_INVALID_ARG;
}
extern "C" tr_status no_model_set_params(tr_context*, no_model*, const float*) {
    return TR_ERR_INVALID_ARG;
}
extern "C" tr_status no_forward(tr_context*, const no_model*, int32_t,
                                const float*, float*) {
    return TR_ERR_INVALID_ARG;
}
extern "C" tr_status no_train_step(tr_context*, no_model*, int32_t, const float*,
                                   const float*, double, double*, float*) {
    return TR_ERR_INVALID_ARG;
}
extern "C" tr_status no_recast_guess(tr_context*, const no_model*, int32_t,
                                     const tr_problem*, double, double, double,
                                     int32_t, float* const*, tr_stats*) {
    return TR_ERR_INVALID_ARG;
}
