// tune.cpp -- runtime choice of the configuration (section 2.3.2 full
// search, extended by the interaction order as in section 4).
//
// Full search: every valid configuration of the search space is run for
// `samples` cycles of R velocity-Verlet steps on the current positions (R
// the rebuild interval); the samples are reduced to one value (the mean,
// the first cycle dropped as warm-up) and the configuration with the
// smallest value is kept (lower index on ties).  The value is the cost of
// one MD step as the integrator runs it with that configuration: re-binning
// (linked cells) or list upkeep and a rebuild every R steps (lists), the
// force kernel and the integrator step.  The steps use a time step of 0, so
// the caller's positions do not move.  Times come from HIP events on the
// context's stream.
//
// Early-stopping search (a cheaper alternative; the paper names full
// search as wasteful, section 2.3.2, and cheaper strategies as future work,
// section 6): the same samples, but a configuration is dropped after its
// warm-up cycle or its first timed cycle when those are well above the best
// value so far, and the configurations are visited most promising first.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <memory>
#include <vector>

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

// The MD step of configuration c as the velocity-Verlet loop runs it: the
// force kernel, the integrator step (fused into the staged Verlet-list
// kernel, or a kernel of its own), the list upkeep between rebuilds and a
// rebuild every R steps, with the host waits of the loop.  The steps take a
// time step of 0 from zero velocities: positions and velocities keep their
// values bit for bit (x + 0 v = x) while every kernel does its usual work.
// One sample is one cycle of R steps (capped at 50), timed with events
// around one step call; sample 0 also builds the structure.
struct Cycles {
    mdlj_ctx *ctx;
    const mdlj_config &c;
    Events ev;
    int R;
    double *v;
    mdlj_status start()
    {
        HIPCHK(ctx, hipEventCreate(&ev.a));
        HIPCHK(ctx, hipEventCreate(&ev.b));
        const int64_t n = ctx->n;
        STCHK(ensure(ctx, ctx->b_tunev, sizeof(double) * 3 * n));
        v = (double *)ctx->b_tunev.p;
        HIPCHK(ctx, hipMemsetAsync(v, 0, sizeof(double) * 3 * n, ctx->stream));
        ctx->cfg = c;
        ctx->built = false;
        ctx->forces_valid = false;
        R = std::max(1, std::min(ctx->rebuild_every, 50));
        return MDLJ_OK;
    }
    // microseconds per step of one more cycle
    mdlj_status sample(double *us)
    {
        const int64_t n = ctx->n;
        HIPCHK(ctx, hipEventRecord(ev.a, ctx->stream));
        STCHK(vv_steps(ctx, v, v + n, v + 2 * n, 0.0, R));
        HIPCHK(ctx, hipEventRecord(ev.b, ctx->stream));
        double t = 0;
        STCHK(elapsed_us(ctx, ev, &t));
        *us = t / R;
        return MDLJ_OK;
    }
};

// Runs `measure_body` with the context's own kernel timing switched off
// (tuning steps are not the caller's) and restores it.  The pruned inner
// list is off too: the measuring steps do not move the particles, so it
// would stay valid through every step of a cycle, where in a run it lasts
// only part of each list period.  Configurations are compared by their
// steps on the full lists; afterwards the lists are marked for a rebuild
// that writes the inner list again.
template <typename F>
mdlj_status untimed(mdlj_ctx *ctx, F &&body)
{
    const bool timing = ctx->timing, prune = ctx->prune;
    ctx->timing = false;
    ctx->prune = false;
    const mdlj_status st = body();
    ctx->timing = timing;
    ctx->prune = prune;
    if (prune) {
        ctx->built = false;
        ctx->inner = 0;
    }
    return st;
}

// Mean microseconds per MD step of configuration c over samples - 1 cycles
// after the warm-up cycle (all of one cycle when samples == 1).
mdlj_status measure(mdlj_ctx *ctx, const mdlj_config &c, int samples, double *out)
{
    return untimed(ctx, [&]() -> mdlj_status {
        Cycles cy{ctx, c, {}, 1, nullptr};
        STCHK(cy.start());
        std::vector<double> t(samples);
        for (int s = 0; s < samples; ++s) STCHK(cy.sample(&t[s]));
        select_config(t.data(), 1, samples, 0, out);
        return MDLJ_OK;
    });
}

// Energy per MD step of configuration c (section 2.3.3): its steps run in
// chunks of whole cycles (each chunk at least 5 ms, so the counter reads
// between chunks idle the GPU little) until the energy counter has been
// refreshed `windows` + 1 times; the mean power between the first and the
// last refresh (joules over their timestamps) times the mean step time of
// the chunks run between them is the energy per step.  *uj = microjoules
// per step, *watts = that mean power, *us = microseconds per step.
mdlj_status measure_energy(mdlj_ctx *ctx, const mdlj_config &c, int windows, double *uj,
                           double *watts, double *us)
{
    return untimed(ctx, [&]() -> mdlj_status {
        Cycles cy{ctx, c, {}, 1, nullptr};
        STCHK(cy.start());
        double warm = 0;
        STCHK(cy.sample(&warm));
        const int per = std::max(1, (int)std::ceil(5000.0 / std::max(warm * cy.R, 1.0)));
        double e = 0, ea = 0, eb = 0;
        uint64_t t = 0, tlast = 0, ta = 0, tb = 0;
        STCHK(energy_read(ctx, &e, &tlast));
        int seen = 0;
        double chunk_us = 0;
        int64_t steps = 0;
        const auto t_start = std::chrono::steady_clock::now();
        while (seen <= windows) {
            double sum = 0;
            for (int k = 0; k < per; ++k) {
                double s_us = 0;
                STCHK(cy.sample(&s_us));
                sum += s_us * cy.R;
            }
            if (seen >= 1) {
                chunk_us += sum;
                steps += (int64_t)per * cy.R;
            }
            STCHK(energy_read(ctx, &e, &t));
            if (t != tlast) {
                if (seen == 0) {
                    ea = e;
                    ta = t;
                } else {
                    eb = e;
                    tb = t;
                }
                ++seen;
                tlast = t;
            }
            const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() -
                                                              t_start).count();
            if (wall > 4.0 + 2.0 * windows)
                return set_err(ctx, MDLJ_ERR_STATE, "the energy counter is not being refreshed");
        }
        if (!(tb > ta) || steps == 0)
            return set_err(ctx, MDLJ_ERR_STATE, "no energy window");
        *watts = (eb - ea) / ((double)(tb - ta) * 1e-9);
        *us = chunk_us / (double)steps;
        *uj = *watts * *us;
        return MDLJ_OK;
    });
}

// The tuner's value of configuration c: microseconds per step (time
// metric) or microjoules per step (energy metric; then also its power).
mdlj_status measure_metric(mdlj_ctx *ctx, const mdlj_config &c, int samples, double *value,
                           double *watts)
{
    *watts = std::numeric_limits<double>::quiet_NaN();
    if (ctx->tune_metric == MDLJ_METRIC_ENERGY) {
        double us = 0;
        return measure_energy(ctx, c, samples, value, watts, &us);
    }
    return measure(ctx, c, samples, value);
}

}  // namespace

// Early-stopping decision of the cheaper search: after sample j of a
// configuration (j = 0 is the warm-up cycle, which also builds the
// structure), whether its next sample is taken, given the best fully
// measured value so far: a configuration whose warm-up cycle is slower than
// warm_factor times the best, or whose first timed cycle is slower than
// (1 + margin) times the best, is dropped.
static bool take_next(int j, double sample, double best, double warm_factor, double margin)
{
    if (!(best < std::numeric_limits<double>::infinity())) return true;
    if (j == 0) return sample <= warm_factor * best;
    if (j == 1) return sample <= (1.0 + margin) * best;
    return true;
}

// The early-stopping search over K configurations visited in `order` (all
// in index order when null), S samples each at most.  fetch(k, j, &x)
// returns sample j of configuration k (called with j = 0, 1, ... in turn;
// x = +inf when the configuration cannot run).  values[k] = the mean of
// samples 1..S-1 of a fully measured configuration (all S when S == 1), the
// last sample of a dropped one (+inf if it cannot run); taken[k] = samples
// used.  Returns the index of the smallest fully measured value (the lower
// index on ties), or -1.
template <typename Fetch>
static mdlj_status search_early(int K, int S, const int *order, double warm_factor,
                                double margin, Fetch &&fetch, double *values, int *taken,
                                int *chosen)
{
    const double inf = std::numeric_limits<double>::infinity();
    int best = -1;
    for (int k = 0; k < K; ++k) {
        values[k] = inf;
        taken[k] = 0;
    }
    std::vector<double> row(S);
    for (int q = 0; q < K; ++q) {
        const int k = order ? order[q] : q;
        const double bv = best >= 0 ? values[best] : inf;
        bool full = true;
        int j = 0;
        while (j < S) {
            double x = inf;
            STCHK(fetch(k, j, &x));
            row[j] = x;
            ++j;
            if (!(x < inf)) {
                full = false;
                break;
            }
            if (j < S && !take_next(j - 1, x, bv, warm_factor, margin)) {
                full = false;
                values[k] = x;
                break;
            }
        }
        taken[k] = j;
        if (!full) continue;
        double v = 0;
        select_config(row.data(), 1, S, 0, &v);
        values[k] = v;
        if (best < 0 || v < values[best] || (v == values[best] && k < best)) best = k;
    }
    *chosen = best;
    return MDLJ_OK;
}

mdlj_status tune_exhaustive(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *best_us)
{
    const mdlj_config saved = ctx->cfg;
    const size_t K = ctx->space.size();
    ctx->tune_us.assign(K, std::numeric_limits<double>::infinity());
    ctx->tune_taken.assign(K, 0);
    ctx->tune_watts.assign(K, std::numeric_limits<double>::quiet_NaN());
    size_t best = K;
    for (size_t k = 0; k < K; ++k) {
        double us = 0, w = 0;
        mdlj_status st = measure_metric(ctx, ctx->space[k], samples, &us, &w);
        if (st == MDLJ_ERR_GEOMETRY || st == MDLJ_ERR_ARG) continue;  // not valid for this box
        if (st != MDLJ_OK) {
            ctx->cfg = saved;
            ctx->built = false;
            return st;
        }
        ctx->tune_us[k] = us;
        ctx->tune_watts[k] = w;
        ctx->tune_taken[k] = samples;
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

// Early-stopping constants of the live search: a configuration is dropped
// when its first timed cycle is more than 10% above the best step time so
// far.  Its warm-up cycle is not scored: besides the structure build it
// carries one-time costs (device buffers allocated the first time a
// structure of that kind is built) that outweigh the steps of small scenes.
constexpr double EARLY_WARM = std::numeric_limits<double>::infinity();
constexpr double EARLY_MARGIN = 0.10;

mdlj_status tune_early(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *best_us)
{
    if (ctx->tune_metric != MDLJ_METRIC_TIME)
        return set_err(ctx, MDLJ_ERR_ARG, "early stopping compares time cycles; the energy metric "
                                          "takes EXHAUSTIVE or FIXED");
    const mdlj_config saved = ctx->cfg;
    const int K = (int)ctx->space.size();
    // most promising first: the network's ranking when one for this search
    // space is loaded, else the search-space order
    std::vector<int> order;
    STCHK(mlp_rank(ctx, order));
    if ((int)order.size() != K) {
        order.resize(K);
        for (int k = 0; k < K; ++k) order[k] = k;
    }
    std::vector<double> values(K);
    std::vector<int> taken(K);
    std::unique_ptr<Cycles> cur;
    const double inf = std::numeric_limits<double>::infinity();
    auto fetch = [&](int k, int j, double *x) -> mdlj_status {
        return untimed(ctx, [&]() -> mdlj_status {
            mdlj_status st = MDLJ_OK;
            if (j == 0) {
                cur.reset(new Cycles{ctx, ctx->space[k], {}, 1, nullptr});
                st = cur->start();
            }
            if (st == MDLJ_OK) st = cur->sample(x);
            if (st == MDLJ_ERR_GEOMETRY || st == MDLJ_ERR_ARG) {  // not valid for this box
                *x = inf;
                ctx->err.clear();
                return MDLJ_OK;
            }
            return st;
        });
    };
    int best = -1;
    const mdlj_status st = search_early(K, samples, order.data(), EARLY_WARM, EARLY_MARGIN, fetch,
                                        values.data(), taken.data(), &best);
    cur.reset();
    ctx->built = false;
    if (st != MDLJ_OK) {
        ctx->cfg = saved;
        return st;
    }
    ctx->tune_us = values;
    ctx->tune_taken = taken;
    if (best < 0) {
        ctx->cfg = saved;
        return set_err(ctx, MDLJ_ERR_GEOMETRY, "no configuration is valid for this system");
    }
    ctx->cfg = ctx->space[best];
    ctx->forces_valid = false;
    ctx->err.clear();
    *chosen = ctx->cfg;
    *best_us = values[best];
    return MDLJ_OK;
}

mdlj_status tune_measure_current(mdlj_ctx *ctx, int samples, double *us)
{
    double w = 0;
    mdlj_status st = measure_metric(ctx, ctx->cfg, samples, us, &w);
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
    case MDLJ_TUNE_EARLY_STOP:
        STCHK(tune_early(ctx, samples, &c, &us));
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

mdlj_status mdlj_tune_select_early(const double *samples, int32_t k, int32_t s,
                                   const int32_t *order, double warm_factor, double margin,
                                   double *values, int32_t *taken, int32_t *chosen)
{
    if (!samples || !values || !taken || !chosen || k < 1 || s < 1 || !(warm_factor >= 1.0) ||
        !(margin >= 0.0) || warm_factor != warm_factor)
        return MDLJ_ERR_ARG;
    if (order) {
        std::vector<char> seen(k, 0);
        for (int32_t q = 0; q < k; ++q) {
            if (order[q] < 0 || order[q] >= k || seen[order[q]]) return MDLJ_ERR_ARG;
            seen[order[q]] = 1;
        }
    }
    auto fetch = [&](int kk, int j, double *x) -> mdlj_status {
        *x = samples[(size_t)kk * s + j];
        if (!(*x == *x)) *x = std::numeric_limits<double>::infinity();
        return MDLJ_OK;
    };
    std::vector<int> tk(k);
    int best = -1;
    STCHK(search_early(k, s, order, warm_factor, margin, fetch, values, tk.data(), &best));
    for (int32_t q = 0; q < k; ++q) taken[q] = tk[q];
    *chosen = best;
    return MDLJ_OK;
}

mdlj_status mdlj_set_tune_metric(mdlj_ctx *ctx, int32_t metric)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (metric != MDLJ_METRIC_TIME && metric != MDLJ_METRIC_ENERGY)
        return set_err(ctx, MDLJ_ERR_ARG, "unknown tuning metric");
    ctx->tune_metric = metric;
    return MDLJ_OK;
}

mdlj_status mdlj_tune_power(const mdlj_ctx *ctx, double *watts, int32_t cap, int32_t *count)
{
    if (!ctx || !count || (cap > 0 && !watts)) return MDLJ_ERR_ARG;
    *count = (int32_t)ctx->tune_watts.size();
    for (int32_t k = 0; k < cap && k < *count; ++k) watts[k] = ctx->tune_watts[k];
    return MDLJ_OK;
}

mdlj_status mdlj_tune_select_energy(const double *us, const double *watts, int32_t k,
                                    double *uj, int32_t *chosen)
{
    if (!us || !watts || !uj || !chosen || k < 1) return MDLJ_ERR_ARG;
    for (int32_t q = 0; q < k; ++q) {
        const double e = us[q] * watts[q];
        uj[q] = (e == e && us[q] > 0 && watts[q] > 0) ? e : std::numeric_limits<double>::infinity();
    }
    *chosen = select_config(uj, k, 1, 0, uj);
    return MDLJ_OK;
}

mdlj_status mdlj_tune_taken(const mdlj_ctx *ctx, int32_t *taken, int32_t cap, int32_t *count)
{
    if (!ctx || !count || (cap > 0 && !taken)) return MDLJ_ERR_ARG;
    *count = (int32_t)ctx->tune_taken.size();
    for (int32_t k = 0; k < cap && k < *count; ++k) taken[k] = ctx->tune_taken[k];
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
