// mlp.hip -- data-driven tuning (the paper's future-work item, section 6):
// a small fully-connected network 8 -> 64 -> 64 -> K (ReLU, softmax over
// the K configurations of the search space) that predicts the fastest
// configuration from eight scene features, trained on timings that the
// exhaustive tuner itself produces.  Forward, backward (cross-entropy) and
// Adam (Kingma & Ba 2015) are hand-written kernels in FP32; when the
// network's confidence (largest softmax probability) is below a threshold
// the tuner falls back to full search.
//
// Parameters are one flat FP32 array:
//   W1[64][8] b1[64] W2[64][64] b2[64] W3[K][64] b3[K]   (row-major [out][in])
// Inputs are z-scored with a stored per-feature mean and deviation.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <random>

#include "internal.h"

namespace {

constexpr int DIN = 8, H1 = 64, H2 = 64, KMAX = 256;

__host__ __device__ inline int64_t n_params(int k)
{
    return (int64_t)H1 * DIN + H1 + (int64_t)H2 * H1 + H2 + (int64_t)k * H2 + k;
}

struct Off {
    int64_t w1, b1, w2, b2, w3, b3;
};

__host__ __device__ inline Off offsets(int k)
{
    Off o;
    o.w1 = 0;
    o.b1 = o.w1 + (int64_t)H1 * DIN;
    o.w2 = o.b1 + H1;
    o.b2 = o.w2 + (int64_t)H2 * H1;
    o.w3 = o.b2 + H2;
    o.b3 = o.w3 + (int64_t)k * H2;
    (void)k;
    return o;
}

// One workgroup of 64 lanes per sample: h1, h2, logits, softmax.
__global__ __launch_bounds__(64) void k_mlp_forward(int B, int K, const float *__restrict__ X,
                                                    const float *__restrict__ w,
                                                    float *__restrict__ h1o,
                                                    float *__restrict__ h2o,
                                                    float *__restrict__ po)
{
    __shared__ float x[DIN], h1[H1], h2[H2], z[KMAX];
    __shared__ float red[2];
    const int s = blockIdx.x, t = threadIdx.x;
    if (s >= B) return;
    const Off o = offsets(K);
    if (t < DIN) x[t] = X[(int64_t)s * DIN + t];
    __syncthreads();
    float a = w[o.b1 + t];
    for (int i = 0; i < DIN; ++i) a += w[o.w1 + t * DIN + i] * x[i];
    h1[t] = a > 0.f ? a : 0.f;
    __syncthreads();
    a = w[o.b2 + t];
    for (int i = 0; i < H1; ++i) a += w[o.w2 + t * H1 + i] * h1[i];
    h2[t] = a > 0.f ? a : 0.f;
    __syncthreads();
    for (int k = t; k < K; k += 64) {
        float zz = w[o.b3 + k];
        for (int i = 0; i < H2; ++i) zz += w[o.w3 + (int64_t)k * H2 + i] * h2[i];
        z[k] = zz;
    }
    __syncthreads();
    if (t == 0) {
        float m = z[0];
        for (int k = 1; k < K; ++k) m = fmaxf(m, z[k]);
        float den = 0.f;
        for (int k = 0; k < K; ++k) den += expf(z[k] - m);
        red[0] = m;
        red[1] = den;
    }
    __syncthreads();
    for (int k = t; k < K; k += 64) po[(int64_t)s * K + k] = expf(z[k] - red[0]) / red[1];
    if (h1o) h1o[(int64_t)s * H1 + t] = h1[t];
    if (h2o) h2o[(int64_t)s * H2 + t] = h2[t];
}

// Per-sample gradient of the mean cross-entropy (1/B included) into row s
// of G, plus the sample's loss term.
__global__ __launch_bounds__(64) void k_mlp_backward(int B, int K, const float *__restrict__ X,
                                                     const int32_t *__restrict__ y,
                                                     const float *__restrict__ w,
                                                     const float *__restrict__ H1v,
                                                     const float *__restrict__ H2v,
                                                     const float *__restrict__ P,
                                                     float *__restrict__ G,
                                                     float *__restrict__ loss)
{
    __shared__ float x[DIN], h1[H1], h2[H2], dz[KMAX], dh2[H2], dh1[H1];
    const int s = blockIdx.x, t = threadIdx.x;
    if (s >= B) return;
    const Off o = offsets(K);
    const int64_t np = n_params(K);
    float *g = G + (int64_t)s * np;
    const int ys = y[s];
    const float invB = 1.0f / (float)B;
    if (t < DIN) x[t] = X[(int64_t)s * DIN + t];
    h1[t] = H1v[(int64_t)s * H1 + t];
    h2[t] = H2v[(int64_t)s * H2 + t];
    for (int k = t; k < K; k += 64) dz[k] = (P[(int64_t)s * K + k] - (k == ys ? 1.f : 0.f)) * invB;
    if (t == 0) loss[s] = -logf(fmaxf(P[(int64_t)s * K + ys], 1e-30f)) * invB;
    __syncthreads();
    // layer 3
    for (int k = t; k < K; k += 64) {
        g[o.b3 + k] = dz[k];
        for (int i = 0; i < H2; ++i) g[o.w3 + (int64_t)k * H2 + i] = dz[k] * h2[i];
    }
    {
        float a = 0.f;
        for (int k = 0; k < K; ++k) a += w[o.w3 + (int64_t)k * H2 + t] * dz[k];
        dh2[t] = h2[t] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // layer 2
    g[o.b2 + t] = dh2[t];
    for (int i = 0; i < H1; ++i) g[o.w2 + t * H1 + i] = dh2[t] * h1[i];
    {
        float a = 0.f;
        for (int k = 0; k < H2; ++k) a += w[o.w2 + k * H1 + t] * dh2[k];
        dh1[t] = h1[t] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // layer 1
    g[o.b1 + t] = dh1[t];
    for (int i = 0; i < DIN; ++i) g[o.w1 + t * DIN + i] = dh1[t] * x[i];
}

// G[p] = sum over samples of G_s[p] (fixed order), loss summed likewise.
__global__ void k_mlp_reduce(int B, int64_t np, const float *__restrict__ Gs,
                             float *__restrict__ G, const float *__restrict__ ls,
                             float *__restrict__ loss)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) {
        float a = 0.f;
        for (int s = 0; s < B; ++s) a += Gs[(int64_t)s * np + p];
        G[p] = a;
    }
    if (p == 0) {
        float a = 0.f;
        for (int s = 0; s < B; ++s) a += ls[s];
        *loss = a;
    }
}

__global__ void k_adam(int64_t np, float *__restrict__ w, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ void k_gather_rows(int B, const int32_t *__restrict__ idx, const float *__restrict__ X,
                              const int32_t *__restrict__ Y, float *__restrict__ xb,
                              int32_t *__restrict__ yb)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const int32_t r = idx[s];
    for (int i = 0; i < DIN; ++i) xb[(int64_t)s * DIN + i] = X[(int64_t)r * DIN + i];
    yb[s] = Y[r];
}

// Scene features: occupancy statistics of a grid of cells of edge >= rc.
__global__ void k_feat_count(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, int nx, int ny, int nz, double lx,
                             double ly, double lz, int32_t *__restrict__ cnt)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p[3] = {x[i], y[i], z[i]};
    const double L[3] = {lx, ly, lz};
    const int nn[3] = {nx, ny, nz};
    int c[3];
    for (int a = 0; a < 3; ++a) {
        const double q = floor(p[a] / L[a]);
        const double m = L[a] * q;
        const double w = p[a] - m;
        const double inv = (double)nn[a] / L[a];
        int k = (int)(w * inv);
        c[a] = k < 0 ? 0 : (k >= nn[a] ? nn[a] - 1 : k);
    }
    atomicAdd(&cnt[c[0] + (int64_t)nx * (c[1] + (int64_t)ny * c[2])], 1);
}

// sum, sum of squares, max and empty count of the cell counts
__global__ __launch_bounds__(256) void k_feat_reduce(int64_t nc, const int32_t *__restrict__ cnt,
                                                     double *__restrict__ out)
{
    __shared__ double s1[256], s2[256], mx[256], em[256];
    double a = 0, b = 0, m = 0, e = 0;
    for (int64_t c = threadIdx.x; c < nc; c += 256) {
        const double v = cnt[c];
        a += v;
        b += v * v;
        m = fmax(m, v);
        e += v == 0 ? 1.0 : 0.0;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    mx[threadIdx.x] = m;
    em[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
            em[threadIdx.x] += em[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s1[0];
        out[1] = s2[0];
        out[2] = mx[0];
        out[3] = em[0];
    }
}

struct MlpDev {
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *gs = nullptr;
    float *x = nullptr, *h1 = nullptr, *h2 = nullptr, *p = nullptr, *ls = nullptr, *loss = nullptr;
    int32_t *y = nullptr;
};

mdlj_status mlp_check(mdlj_ctx *ctx)
{
    if (ctx->mlp_k < 1 || (int64_t)ctx->mlp_w.size() != n_params(ctx->mlp_k))
        return set_err(ctx, MDLJ_ERR_STATE, "network not initialised");
    return MDLJ_OK;
}

// forward on the device for B already-normalised rows (host in, host out)
mdlj_status forward_host(mdlj_ctx *ctx, const float *xn, int B, float *probs)
{
    const int K = ctx->mlp_k;
    const int64_t np = n_params(K);
    STCHK(ensure(ctx, ctx->b_mlp, sizeof(float) * (np + (int64_t)B * (DIN + K))));
    float *w = (float *)ctx->b_mlp.p;
    float *x = w + np;
    float *p = x + (int64_t)B * DIN;
    HIPCHK(ctx, hipMemcpyAsync(w, ctx->mlp_w.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(x, xn, sizeof(float) * B * DIN, hipMemcpyHostToDevice, ctx->stream));
    k_mlp_forward<<<B, 64, 0, ctx->stream>>>(B, K, x, w, nullptr, nullptr, p);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(probs, p, sizeof(float) * B * K, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDLJ_OK;
}

void normalise(const mdlj_ctx *ctx, const float *x, int n, std::vector<float> &out)
{
    out.resize((size_t)n * DIN);
    for (int s = 0; s < n; ++s)
        for (int i = 0; i < DIN; ++i)
            out[(size_t)s * DIN + i] = (x[(size_t)s * DIN + i] - ctx->mlp_mean[i]) / ctx->mlp_std[i];
}

}  // namespace

mdlj_status features_dev(mdlj_ctx *ctx, float *f8)
{
    const double *L = ctx->box;
    const double rc = ctx->rc;
    int nn[3];
    for (int a = 0; a < 3; ++a) nn[a] = std::max(1, (int)floor(L[a] / rc));
    const int64_t nc = (int64_t)nn[0] * nn[1] * nn[2];
    STCHK(ensure(ctx, ctx->b_feat, sizeof(int32_t) * nc + 64));
    STCHK(ensure(ctx, ctx->b_flags, sizeof(int32_t) * 64));
    int32_t *cnt = (int32_t *)ctx->b_feat.p;
    double *out = (double *)ctx->b_flags.p + 20;
    HIPCHK(ctx, hipMemsetAsync(cnt, 0, sizeof(int32_t) * nc, ctx->stream));
    k_feat_count<<<ceil_div(ctx->n, 256), 256, 0, ctx->stream>>>(ctx->n, ctx->x, ctx->y, ctx->z,
                                                               nn[0], nn[1], nn[2], L[0], L[1],
                                                               L[2], cnt);
    k_feat_reduce<<<1, 256, 0, ctx->stream>>>(nc, cnt, out);
    HIPCHK(ctx, hipGetLastError());
    double h[4];
    HIPCHK(ctx, hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const double N = (double)ctx->n;
    const double vol = L[0] * L[1] * L[2];
    const double rho = N / vol;
    double smax = 0;
    for (int s = 0; s < ctx->nspec; ++s) smax = std::max(smax, ctx->sig[s]);
    const double mean = h[0] / (double)nc;
    const double var = std::max(0.0, h[1] / (double)nc - mean * mean);
    f8[0] = (float)log10(N);
    f8[1] = (float)rho;
    f8[2] = (float)(rc / smax);
    f8[3] = (float)ctx->nspec;
    f8[4] = (float)(rho * 4.18879020478639 * rc * rc * rc);
    f8[5] = (float)(mean > 0 ? sqrt(var) / mean : 0.0);
    f8[6] = (float)(h[3] / (double)nc);
    f8[7] = (float)(mean > 0 ? h[2] / mean : 0.0);
    return MDLJ_OK;
}

// A network covers the first mlp_k configurations of the search space
// (configurations added to the space after it was trained come after those
// it knows, so its output k still names space[k]).
static bool mlp_usable(const mdlj_ctx *ctx)
{
    return ctx->mlp_loaded && ctx->mlp_k >= 1 && ctx->mlp_k <= (int)ctx->space.size();
}

mdlj_status mlp_rank(mdlj_ctx *ctx, std::vector<int> &order)
{
    order.clear();
    if (!mlp_usable(ctx)) return MDLJ_OK;
    float f[DIN];
    STCHK(features_dev(ctx, f));
    std::vector<float> xn;
    normalise(ctx, f, 1, xn);
    std::vector<float> p(ctx->mlp_k);
    STCHK(forward_host(ctx, xn.data(), 1, p.data()));
    order.resize(ctx->mlp_k);
    for (int k = 0; k < ctx->mlp_k; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p[a] > p[b]; });
    // configurations the network does not know, after those it ranks
    for (int k = ctx->mlp_k; k < (int)ctx->space.size(); ++k) order.push_back(k);
    return MDLJ_OK;
}

mdlj_status tune_learned(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *us)
{
    // the network predicts the fastest configuration: under the energy
    // metric the full search decides
    if (!mlp_usable(ctx) || ctx->tune_metric != MDLJ_METRIC_TIME)
        return tune_exhaustive(ctx, samples, chosen, us);
    float f[DIN];
    STCHK(features_dev(ctx, f));
    std::vector<float> xn;
    normalise(ctx, f, 1, xn);
    std::vector<float> p(ctx->mlp_k);
    STCHK(forward_host(ctx, xn.data(), 1, p.data()));
    int best = (int)(std::max_element(p.begin(), p.end()) - p.begin());
    ctx->mlp_last_conf = p[best];
    if (p[best] < ctx->mlp_threshold) {
        ctx->mlp_fallbacks++;
        return tune_exhaustive(ctx, samples, chosen, us);
    }
    const mdlj_config saved = ctx->cfg;
    ctx->cfg = ctx->space[best];
    mdlj_status st = tune_measure_current(ctx, samples, us);
    if (st == MDLJ_ERR_GEOMETRY || st == MDLJ_ERR_ARG) {
        // predicted configuration not valid here: full search decides
        ctx->cfg = saved;
        ctx->mlp_fallbacks++;
        return tune_exhaustive(ctx, samples, chosen, us);
    }
    STCHK(st);
    *chosen = ctx->cfg;
    return MDLJ_OK;
}

extern "C" {

mdlj_status mdlj_features(mdlj_ctx *ctx, float *features8)
{
    if (!ctx || !features8) return MDLJ_ERR_ARG;
    if (!ctx->box_set || !(ctx->rc > 0)) return set_err(ctx, MDLJ_ERR_STATE, "box or cutoff not set");
    return features_dev(ctx, features8);
}

mdlj_status mdlj_mlp_init(mdlj_ctx *ctx, int32_t k, uint64_t seed)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (k < 1 || k > KMAX) return set_err(ctx, MDLJ_ERR_ARG, "class count must be 1..256");
    ctx->mlp_k = k;
    ctx->mlp_w.assign(n_params(k), 0.f);
    const Off o = offsets(k);
    std::mt19937_64 rng(seed);
    auto he = [&](int64_t off, int64_t count, int fan_in) {
        std::normal_distribution<double> nd(0.0, sqrt(2.0 / fan_in));
        for (int64_t i = 0; i < count; ++i) ctx->mlp_w[off + i] = (float)nd(rng);
    };
    he(o.w1, (int64_t)H1 * DIN, DIN);
    he(o.w2, (int64_t)H2 * H1, H1);
    he(o.w3, (int64_t)k * H2, H2);
    for (int i = 0; i < DIN; ++i) {
        ctx->mlp_mean[i] = 0.f;
        ctx->mlp_std[i] = 1.f;
    }
    ctx->mlp_loaded = true;
    ctx->mlp_adam_t = 0;
    ctx->mlp_m.assign(ctx->mlp_w.size(), 0.f);
    ctx->mlp_v.assign(ctx->mlp_w.size(), 0.f);
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_set_norm(mdlj_ctx *ctx, const float *mean8, const float *std8)
{
    if (!ctx || !mean8 || !std8) return MDLJ_ERR_ARG;
    for (int i = 0; i < DIN; ++i) {
        if (!(std8[i] > 0) || !isfinite(mean8[i])) return set_err(ctx, MDLJ_ERR_ARG, "bad normalisation");
        ctx->mlp_mean[i] = mean8[i];
        ctx->mlp_std[i] = std8[i];
    }
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_get_params(const mdlj_ctx *ctx, float *w, int64_t cap, int64_t *count,
                                int32_t *k)
{
    if (!ctx || !count) return MDLJ_ERR_ARG;
    *count = (int64_t)ctx->mlp_w.size();
    if (k) *k = ctx->mlp_k;
    if (w) std::copy(ctx->mlp_w.begin(), ctx->mlp_w.begin() + std::min<int64_t>(cap, *count), w);
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_set_params(mdlj_ctx *ctx, const float *w, int64_t count, int32_t k)
{
    if (!ctx || !w || k < 1 || k > KMAX || count != n_params(k)) return MDLJ_ERR_ARG;
    ctx->mlp_k = k;
    ctx->mlp_w.assign(w, w + count);
    ctx->mlp_m.assign(count, 0.f);
    ctx->mlp_v.assign(count, 0.f);
    ctx->mlp_adam_t = 0;
    ctx->mlp_loaded = true;
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_predict(mdlj_ctx *ctx, const float *x, int32_t n, float *probs)
{
    if (!ctx || !x || !probs || n < 1) return MDLJ_ERR_ARG;
    STCHK(mlp_check(ctx));
    std::vector<float> xn;
    normalise(ctx, x, n, xn);
    return forward_host(ctx, xn.data(), n, probs);
}

// Loss and gradient of the current parameters on n raw (un-normalised
// by the network, i.e. used as given) input rows.
mdlj_status mdlj_mlp_loss_grad(mdlj_ctx *ctx, const float *x, const int32_t *labels, int32_t n,
                               float *grad, float *loss)
{
    if (!ctx || !x || !labels || !grad || !loss || n < 1) return MDLJ_ERR_ARG;
    STCHK(mlp_check(ctx));
    const int K = ctx->mlp_k;
    for (int s = 0; s < n; ++s)
        if (labels[s] < 0 || labels[s] >= K) return set_err(ctx, MDLJ_ERR_ARG, "label out of range");
    const int64_t np = n_params(K);
    const int64_t B = n;
    const size_t floats = np * 2 + B * np + B * (DIN + H1 + H2 + K + 1) + 1;
    STCHK(ensure(ctx, ctx->b_mlp, sizeof(float) * floats + sizeof(int32_t) * B));
    float *w = (float *)ctx->b_mlp.p;
    float *g = w + np;
    float *gs = g + np;
    float *xd = gs + B * np;
    float *h1 = xd + B * DIN;
    float *h2 = h1 + B * H1;
    float *p = h2 + B * H2;
    float *ls = p + B * K;
    float *ld = ls + B;
    int32_t *yd = (int32_t *)(ld + 1);
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipMemcpyAsync(w, ctx->mlp_w.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(xd, x, sizeof(float) * B * DIN, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(yd, labels, sizeof(int32_t) * B, hipMemcpyHostToDevice, st));
    k_mlp_forward<<<B, 64, 0, st>>>((int)B, K, xd, w, h1, h2, p);
    k_mlp_backward<<<B, 64, 0, st>>>((int)B, K, xd, yd, w, h1, h2, p, gs, ls);
    k_mlp_reduce<<<ceil_div(np, 256), 256, 0, st>>>((int)B, np, gs, g, ls, ld);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(grad, g, sizeof(float) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return MDLJ_OK;
}

// Adam training on the device: epochs over n rows (raw features, normalised
// here with the stored mean/deviation), minibatches of `batch` rows in a
// seeded shuffled order.  Continues the Adam moments of earlier calls.
mdlj_status mdlj_mlp_train(mdlj_ctx *ctx, const float *x, const int32_t *labels, int32_t n,
                           int32_t epochs, int32_t batch, double lr, uint64_t seed,
                           double *final_loss)
{
    if (!ctx || !x || !labels || n < 1 || epochs < 0 || batch < 1 || !(lr > 0))
        return MDLJ_ERR_ARG;
    STCHK(mlp_check(ctx));
    const int K = ctx->mlp_k;
    for (int s = 0; s < n; ++s)
        if (labels[s] < 0 || labels[s] >= K) return set_err(ctx, MDLJ_ERR_ARG, "label out of range");
    const int64_t np = n_params(K);
    const int64_t B = std::min<int64_t>(batch, n);
    std::vector<float> xn;
    normalise(ctx, x, n, xn);
    const size_t floats = np * 5 + B * np + B * (DIN + H1 + H2 + K + 1) + 1 + (size_t)n * DIN;
    STCHK(ensure(ctx, ctx->b_mlp, sizeof(float) * floats + sizeof(int32_t) * (2 * B + n)));
    float *w = (float *)ctx->b_mlp.p;
    float *m = w + np;
    float *v = m + np;
    float *g = v + np;
    float *gs = g + np;
    float *xb = gs + B * np;
    float *h1 = xb + B * DIN;
    float *h2 = h1 + B * H1;
    float *p = h2 + B * H2;
    float *ls = p + B * K;
    float *ld = ls + B;
    float *X = ld + 1;
    int32_t *yb = (int32_t *)(X + (size_t)n * DIN);
    int32_t *Y = yb + B;
    int32_t *idx = Y + n;
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipMemcpyAsync(w, ctx->mlp_w.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m, ctx->mlp_m.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(v, ctx->mlp_v.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(X, xn.data(), sizeof(float) * n * DIN, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(Y, labels, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float hl = 0.f;
    double epoch_loss = 0.0;
    std::vector<int32_t> hidx((size_t)B);
    for (int e = 0; e < epochs; ++e) {
        std::shuffle(order.begin(), order.end(), rng);
        epoch_loss = 0.0;
        int nb = 0;
        for (int64_t b0 = 0; b0 + B <= n; b0 += B) {
            HIPCHK(ctx, hipMemcpyAsync(idx, order.data() + b0, sizeof(int32_t) * B,
                                       hipMemcpyHostToDevice, st));
            k_gather_rows<<<ceil_div(B, 64), 64, 0, st>>>((int)B, idx, X, Y, xb, yb);
            k_mlp_forward<<<B, 64, 0, st>>>((int)B, K, xb, w, h1, h2, p);
            k_mlp_backward<<<B, 64, 0, st>>>((int)B, K, xb, yb, w, h1, h2, p, gs, ls);
            k_mlp_reduce<<<ceil_div(np, 256), 256, 0, st>>>((int)B, np, gs, g, ls, ld);
            ctx->mlp_adam_t++;
            const int t = ctx->mlp_adam_t;
            const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
            k_adam<<<ceil_div(np, 256), 256, 0, st>>>(np, w, g, m, v, (float)lr, b1, b2, eps, c1, c2);
            HIPCHK(ctx, hipGetLastError());
            HIPCHK(ctx, hipMemcpyAsync(&hl, ld, sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(ctx, hipStreamSynchronize(st));
            epoch_loss += hl;
            ++nb;
        }
        if (nb) epoch_loss /= nb;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->mlp_w.data(), w, sizeof(float) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(ctx->mlp_m.data(), m, sizeof(float) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(ctx->mlp_v.data(), v, sizeof(float) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (final_loss) *final_loss = epoch_loss;
    return MDLJ_OK;
}

// File: "MDLJMLP1", int32 K, int32 din, int32 h1, int32 h2, float mean[8],
// float std[8], float params[n_params(K)]  (little-endian)
mdlj_status mdlj_mlp_save(const mdlj_ctx *ctx, const char *path)
{
    if (!ctx || !path) return MDLJ_ERR_ARG;
    if (ctx->mlp_k < 1) return MDLJ_ERR_STATE;
    FILE *f = fopen(path, "wb");
    if (!f) return MDLJ_ERR_NOTFOUND;
    const int32_t hdr[4] = {ctx->mlp_k, DIN, H1, H2};
    bool ok = fwrite("MDLJMLP1", 1, 8, f) == 8 && fwrite(hdr, sizeof(int32_t), 4, f) == 4 &&
              fwrite(ctx->mlp_mean, sizeof(float), DIN, f) == DIN &&
              fwrite(ctx->mlp_std, sizeof(float), DIN, f) == DIN &&
              fwrite(ctx->mlp_w.data(), sizeof(float), ctx->mlp_w.size(), f) == ctx->mlp_w.size();
    fclose(f);
    return ok ? MDLJ_OK : MDLJ_ERR_NOTFOUND;
}

mdlj_status mdlj_mlp_load(mdlj_ctx *ctx, const char *path)
{
    if (!ctx || !path) return MDLJ_ERR_ARG;
    FILE *f = fopen(path, "rb");
    if (!f) return set_err(ctx, MDLJ_ERR_NOTFOUND, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[4];
    float mean[DIN], sd[DIN];
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "MDLJMLP1", 8) == 0 &&
              fread(hdr, sizeof(int32_t), 4, f) == 4 && hdr[1] == DIN && hdr[2] == H1 &&
              hdr[3] == H2 && hdr[0] >= 1 && hdr[0] <= KMAX &&
              fread(mean, sizeof(float), DIN, f) == DIN && fread(sd, sizeof(float), DIN, f) == DIN;
    std::vector<float> w;
    if (ok) {
        w.resize(n_params(hdr[0]));
        ok = fread(w.data(), sizeof(float), w.size(), f) == w.size();
    }
    fclose(f);
    if (!ok) return set_err(ctx, MDLJ_ERR_ARG, "not a network file of this library");
    STCHK(mdlj_mlp_set_params(ctx, w.data(), (int64_t)w.size(), hdr[0]));
    STCHK(mdlj_mlp_set_norm(ctx, mean, sd));
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_set_threshold(mdlj_ctx *ctx, double threshold)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!(threshold >= 0.0 && threshold <= 1.0)) return set_err(ctx, MDLJ_ERR_ARG, "threshold must be in [0, 1]");
    ctx->mlp_threshold = threshold;
    return MDLJ_OK;
}

mdlj_status mdlj_mlp_stats(const mdlj_ctx *ctx, double *last_confidence, int64_t *fallbacks)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (last_confidence) *last_confidence = ctx->mlp_last_conf;
    if (fallbacks) *fallbacks = ctx->mlp_fallbacks;
    return MDLJ_OK;
}

}  // extern "C"
