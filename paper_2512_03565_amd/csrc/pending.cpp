// pending.cpp -- entry points whose implementation lands in later files.
#include "internal.h"

mdlj_status vl_build(mdlj_ctx *ctx, const mdlj_config &) { return set_err(ctx, MDLJ_ERR_ARG, "Verlet lists not available"); }
mdlj_status vl_forces(mdlj_ctx *ctx, const mdlj_config &, bool, ForceOut &, int64_t *) { return set_err(ctx, MDLJ_ERR_ARG, "Verlet lists not available"); }
mdlj_status vcl_build(mdlj_ctx *ctx, const mdlj_config &) { return set_err(ctx, MDLJ_ERR_ARG, "cluster lists not available"); }
mdlj_status vcl_forces(mdlj_ctx *ctx, const mdlj_config &, bool, ForceOut &, int64_t *) { return set_err(ctx, MDLJ_ERR_ARG, "cluster lists not available"); }

extern "C" {
mdlj_status mdlj_tune(mdlj_ctx *ctx, int32_t, int32_t, mdlj_config *, double *) { return ctx ? set_err(ctx, MDLJ_ERR_STATE, "tuner not available") : MDLJ_ERR_ARG; }
mdlj_status mdlj_tune_results(const mdlj_ctx *ctx, double *, int32_t, int32_t *) { return ctx ? MDLJ_ERR_STATE : MDLJ_ERR_ARG; }
mdlj_status mdlj_step_vv(mdlj_ctx *ctx, double *, double *, double *, double, int32_t) { return ctx ? set_err(ctx, MDLJ_ERR_STATE, "integrator not available") : MDLJ_ERR_ARG; }
mdlj_status mdlj_features(mdlj_ctx *ctx, float *) { return ctx ? set_err(ctx, MDLJ_ERR_STATE, "features not available") : MDLJ_ERR_ARG; }
mdlj_status mdlj_mlp_load(mdlj_ctx *ctx, const char *) { return ctx ? set_err(ctx, MDLJ_ERR_STATE, "network not available") : MDLJ_ERR_ARG; }
mdlj_status mdlj_mlp_save(const mdlj_ctx *ctx, const char *) { return ctx ? MDLJ_ERR_STATE : MDLJ_ERR_ARG; }
mdlj_status mdlj_mlp_set_threshold(mdlj_ctx *ctx, double t) { if (!ctx) return MDLJ_ERR_ARG; ctx->mlp_threshold = t; return MDLJ_OK; }
}
