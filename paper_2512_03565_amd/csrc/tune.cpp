// tune.cpp -- runtime choice of the configuration (section 2.3.2 full
// search, extended by the interaction order as in section 4).
//
// Full search: every valid configuration of the search space is run for
// `samples` force evaluations on the current positions; the samples are
// reduced to one value (the mean, first sample dropped as warm-up) and the
// configuration with the smallest value is kept (lower index on ties).  The
// value is the amortised cost of one MD step with that configuration:
//   linked cells:  re-binning + force kernel          (every step)
//   lists:         force kernel + (R-1)/R * upkeep + rebuild / R
// where R is the rebuild interval and upkeep the per-step displacement
// check and record refresh.  Times come from HIP events on the context's
// stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <limits>

#include "internal.h"

// Reduce S samples of each of K configurations (row-major [K][S], +inf or
// NaN for a configuration that cannot run) to one value each -- the mean
// with the first sample dropped as warm-up (mode 0, all S when S == 1) or
// the minimum (mode 1) -- and pick the smallest, lower index on ties.
// Returns the chosen index or -1 when none is finite.
static int select_config(const double *samples, int K, int S, int mode, double *values)
{
    int best = -1;
    for (int k = 0; k < K; ++k) {
        const double *row = samples + (size_t)k * S;
        double v;
        if (mode == 1) {
            v = std::numeric_limits<double>::infinity();
            for (int s = 0; s < S; ++s) v = row[s] < v ? row[s] : v;
        } else {
            const int first = S > 1 ? 1 : 0;
            double sum = 0;
            for (int s = first; s < S; ++s) sum += row[s];
            v = sum / (S - first);
        }
        if (!(v == v)) v = std::numeric_limits<double>::infinity();  // NaN -> cannot run
        values[k] = v;
        if (v < std::numeric_limits<double>::infinity() && (best < 0 || v < values[best])) best = k;
    }
    return best;
}

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

mdlj_status elapsed_us(mdlj_ctx *ctx, Events &ev, double *us)
{
    HIPCHK(ctx, hipEventSynchronize(ev.b));
    float ms = 0;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ev.a, ev.b));
    *us = 1e3 * ms;
    return MDLJ_OK;
}

// Amortised microseconds per step of configuration c (positions fixed).
mdlj_status measure(mdlj_ctx *ctx, const mdlj_config &c, int samples, double *out)
{
    Events ev;
    HIPCHK(ctx, hipEventCreate(&ev.a));
    HIPCHK(ctx, hipEventCreate(&ev.b));
    ctx->cfg = c;
    ctx->built = false;
    bool rebuilt = false;
    double build_us = 0, upkeep_us = 0;
    HIPCHK(ctx, hipEventRecord(ev.a, ctx->stream));
    STCHK(prepare(ctx, c, true, &rebuilt));
    HIPCHK(ctx, hipEventRecord(ev.b, ctx->stream));
    STCHK(elapsed_us(ctx, ev, &build_us));
    if (c.nbr_algo != MDLJ_NBR_LC) {
        // per-step upkeep between rebuilds: displacement check + refresh
        HIPCHK(ctx, hipEventRecord(ev.a, ctx->stream));
        bool far = false;
        STCHK(moved_too_far(ctx, &far));
        STCHK(refresh_records(ctx));
        HIPCHK(ctx, hipEventRecord(ev.b, ctx->stream));
        STCHK(elapsed_us(ctx, ev, &upkeep_us));
    }
    std::vector<double> t(samples);
    for (int s = 0; s < samples; ++s) {
        ForceOut fo;
        int64_t nb = 0;
        HIPCHK(ctx, hipEventRecord(ev.a, ctx->stream));
        STCHK(run_force_kernel(ctx, c, false, fo, &nb));
        if (needs_fold(c)) STCHK(fold_forces(ctx, fo));
        STCHK(unpermute_forces(ctx, fo, ctx->fx, ctx->fy, ctx->fz));
        HIPCHK(ctx, hipEventRecord(ev.b, ctx->stream));
        STCHK(elapsed_us(ctx, ev, &t[s]));
    }
    double force_us = 0;
    select_config(t.data(), 1, samples, 0, &force_us);
    if (c.nbr_algo == MDLJ_NBR_LC) {
        *out = force_us + build_us;
    } else {
        const double R = ctx->rebuild_every;
        *out = force_us + upkeep_us * (R - 1.0) / R + build_us / R;
    }
    ctx->forces_valid = true;
    ctx->steps_since_build = 1;
    return MDLJ_OK;
}

}  // namespace

mdlj_status tune_exhaustive(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *best_us)
{
    const mdlj_config saved = ctx->cfg;
    const size_t K = ctx->space.size();
    ctx->tune_us.assign(K, std::numeric_limits<double>::infinity());
    size_t best = K;
    for (size_t k = 0; k < K; ++k) {
        double us = 0;
        mdlj_status st = measure(ctx, ctx->space[k], samples, &us);
        if (st == MDLJ_ERR_GEOMETRY || st == MDLJ_ERR_ARG) continue;  // not valid for this box
        if (st != MDLJ_OK) {
            ctx->cfg = saved;
            ctx->built = false;
            return st;
        }
        ctx->tune_us[k] = us;
        if (best == K || us < ctx->tune_us[best]) best = k;
    }
    ctx->built = false;
    if (best == K) {
        ctx->cfg = saved;
        return set_err(ctx, MDLJ_ERR_GEOMETRY, "no configuration is valid for this system");
    }
    ctx->cfg = ctx->space[best];
    ctx->forces_valid = false;
    ctx->err.clear();
    *chosen = ctx->cfg;
    *best_us = ctx->tune_us[best];
    return MDLJ_OK;
}

mdlj_status tune_measure_current(mdlj_ctx *ctx, int samples, double *us)
{
    mdlj_status st = measure(ctx, ctx->cfg, samples, us);
    ctx->built = false;
    ctx->forces_valid = false;
    return st;
}

extern "C" {

mdlj_status mdlj_tune(mdlj_ctx *ctx, int32_t mode, int32_t samples, mdlj_config *chosen,
                      double *step_us)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (samples < 1 || samples > 1000) return set_err(ctx, MDLJ_ERR_ARG, "samples must be 1..1000");
    mdlj_config c = ctx->cfg;
    double us = 0;
    switch (mode) {
    case MDLJ_TUNE_FIXED:
        STCHK(tune_measure_current(ctx, samples, &us));
        break;
    case MDLJ_TUNE_EXHAUSTIVE:
        STCHK(tune_exhaustive(ctx, samples, &c, &us));
        break;
    case MDLJ_TUNE_LEARNED:
        STCHK(tune_learned(ctx, samples, &c, &us));
        break;
    default:
        return set_err(ctx, MDLJ_ERR_ARG, "unknown tuning mode");
    }
    if (chosen) *chosen = ctx->cfg;
    if (step_us) *step_us = us;
    return MDLJ_OK;
}

mdlj_status mdlj_tune_select(const double *samples, int32_t k, int32_t s, int32_t mode,
                             double *values, int32_t *chosen)
{
    if (!samples || !values || !chosen || k < 1 || s < 1 || (mode != 0 && mode != 1))
        return MDLJ_ERR_ARG;
    *chosen = select_config(samples, k, s, mode, values);
    return MDLJ_OK;
}

mdlj_status mdlj_retune_needed(const float *before8, const float *now8, double threshold,
                               int32_t *needed)
{
    if (!before8 || !now8 || !needed || !(threshold >= 0)) return MDLJ_ERR_ARG;
    // density (feature 1) and cell-occupancy spread (feature 5) are the
    // quantities whose change moves the optimum (section 5)
    const int idx[2] = {1, 5};
    *needed = 0;
    for (int q = 0; q < 2; ++q) {
        const double a = before8[idx[q]], b = now8[idx[q]];
        const double den = fabs(a) > 1e-12 ? fabs(a) : 1e-12;
        if (fabs(b - a) / den > threshold) *needed = 1;
    }
    return MDLJ_OK;
}

mdlj_status mdlj_tune_results(const mdlj_ctx *ctx, double *us, int32_t cap, int32_t *count)
{
    if (!ctx || !count || (cap > 0 && !us)) return MDLJ_ERR_ARG;
    *count = (int32_t)ctx->tune_us.size();
    for (int32_t k = 0; k < cap && k < *count; ++k) us[k] = ctx->tune_us[k];
    return MDLJ_OK;
}

}  // extern "C"
