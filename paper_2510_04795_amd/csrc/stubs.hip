// Entry points whose device code is not built yet.
#include "runtime.h"
using namespace oz;
extern "C" {
int heff_plan_create(ozaki_ctx, heff_plan *out, const heff_layout *, const double *, const double *,
                     int32_t, const heff_triple *, const double *, int, int, void *) {
    if (out) *out = nullptr;
    return fail(OZ_ERR_UNSUPPORTED, "heff_plan_create: not built");
}
int heff_apply(heff_plan, const double *, double *, void *) { return fail(OZ_ERR_UNSUPPORTED, "not built"); }
int64_t heff_vector_length(heff_plan) { return -1; }
double heff_flops(heff_plan) { return 0.0; }
int heff_plan_destroy(heff_plan) { return OZ_OK; }
int davidson_create(ozaki_ctx, davidson *out, heff_plan, const double *, const double *, int, double, int, void *) {
    if (out) *out = nullptr;
    return fail(OZ_ERR_UNSUPPORTED, "davidson_create: not built");
}
int davidson_step(davidson, davidson_info *, void *) { return fail(OZ_ERR_UNSUPPORTED, "not built"); }
int davidson_get_vector(davidson, double *, void *) { return fail(OZ_ERR_UNSUPPORTED, "not built"); }
int davidson_destroy(davidson) { return OZ_OK; }
}
