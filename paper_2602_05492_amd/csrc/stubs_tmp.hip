#include "common.hpp"
extern "C" {
int bem_jtj(bem_ctx* ctx, const double*, int32_t, const double*, int64_t, const void*, double*, double*, bem_gram, bem_prec, hipStream_t)
{ return bem::set_error(ctx, BEM_EINVAL, "not yet"); }
int lm_step(bem_ctx* ctx, double*, int32_t, const double*, int64_t, const double*, bem_lm_state*, bem_gram, bem_prec, hipStream_t)
{ return bem::set_error(ctx, BEM_EINVAL, "not yet"); }
int bem_jacobian(bem_ctx* ctx, const double*, int32_t, const double*, int64_t, double*, hipStream_t)
{ return bem::set_error(ctx, BEM_EINVAL, "not yet"); }
}
