// Host side of the learned spectral filter: trainer (statistics of method-generated
// frames, FP32 training steps with Adam on the GPU) and stand-alone BF16 inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "learn_internal.h"

using namespace safr;

namespace safr {
safr_status set_error(safr_status st, const char* msg);
}

namespace {

safr_status lfail(safr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return set_error(st, buf);
}

#define L_TRY(expr)                                                                           \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) return lfail(SAFR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

}  // namespace

struct safr_trainer {
    int M = 0, G = 0, L = 0, r = 0, Kh = 0, stride = 0;
    size_t H = 0;
    LearnFreq fq{};
    LearnFreq* fq_dev = nullptr;
    float* amp = nullptr;
    double Z = 0.0;
    float noise_scale = 0.f;
    int max_frames = 0, nframes = 0;
    float* stats = nullptr;
    float* eta = nullptr;
    float* params = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int step = 0;
    float* act = nullptr;
    size_t act_rows = 0;
    float* partials = nullptr;
    int chunks_cap = 0;
    float* loss_part = nullptr;
    int loss_cap = 0;
    int* frames = nullptr;
    int frames_cap = 0;
    float* grad = nullptr;
};

namespace {

void free_trainer(safr_trainer* t) {
    if (!t) return;
    (void)hipFree(t->fq.U);
    (void)hipFree(t->fq.V);
    (void)hipFree(t->fq.inv_sigma);
    (void)hipFree(t->fq.feat);
    (void)hipFree(t->fq.s);
    (void)hipFree(t->fq.ph);
    (void)hipFree(t->fq.mult);
    (void)hipFree(t->fq_dev);
    (void)hipFree(t->amp);
    (void)hipFree(t->stats);
    (void)hipFree(t->eta);
    (void)hipFree(t->params);
    (void)hipFree(t->m);
    (void)hipFree(t->v);
    (void)hipFree(t->act);
    (void)hipFree(t->partials);
    (void)hipFree(t->loss_part);
    (void)hipFree(t->frames);
    (void)hipFree(t->grad);
    delete t;
}

// one forward/backward over the batch; partial gradients in t->partials, per-block losses in t->loss_part
safr_status run_batch(safr_trainer* t, int nb, const int* frames, hipStream_t s, int* chunks_out, int* blocks_out) {
    for (int i = 0; i < nb; ++i)
        if (frames[i] < 0 || frames[i] >= t->nframes) return lfail(SAFR_ERR_ARG, "frame index %d out of range", frames[i]);
    if (nb > t->frames_cap) {
        (void)hipFree(t->frames);
        t->frames = nullptr;
        L_TRY(hipMalloc(&t->frames, nb * sizeof(int)));
        t->frames_cap = nb;
    }
    L_TRY(hipMemcpy(t->frames, frames, nb * sizeof(int), hipMemcpyHostToDevice));
    const size_t rows = (size_t)nb * t->H * t->r;
    if (rows > t->act_rows) {
        (void)hipFree(t->act);
        t->act = nullptr;
        L_TRY(hipMalloc(&t->act, rows * ACT_PLANES * sizeof(float)));
        t->act_rows = rows;
    }
    const int threads = 128;
    const int blocks = (int)((nb * t->H + threads - 1) / threads);
    if (blocks > t->loss_cap) {
        (void)hipFree(t->loss_part);
        t->loss_part = nullptr;
        L_TRY(hipMalloc(&t->loss_part, blocks * sizeof(float)));
        t->loss_cap = blocks;
    }
    MlpRowsArgs ra{};
    ra.params = t->params;
    ra.feat = t->fq.feat;
    ra.mult = t->fq.mult;
    ra.stats = t->stats;
    ra.eta = t->eta;
    ra.frames = t->frames;
    ra.act = t->act;
    ra.loss_part = t->loss_part;
    ra.scale = (float)(1.0 / (t->Z * nb));
    ra.nb = nb;
    ra.r = t->r;
    ra.stride = t->stride;
    ra.H = t->H;
    const size_t lds = mlp_rows_lds_bytes(threads);
    allow_large_lds(reinterpret_cast<const void*>(&mlp_rows_kernel));
    hipLaunchKernelGGL(mlp_rows_kernel, dim3(blocks), dim3(threads), lds, s, ra);
    L_TRY(hipGetLastError());
    const int chunks = (int)std::min<size_t>(256, (rows + 1023) / 1024);
    if (chunks > t->chunks_cap) {
        (void)hipFree(t->partials);
        t->partials = nullptr;
        L_TRY(hipMalloc(&t->partials, (size_t)chunks * 8705 * sizeof(float)));
        t->chunks_cap = chunks;
    }
    MlpGradArgs ga{};
    ga.act = t->act;
    ga.partials = t->partials;
    ga.rows = rows;
    ga.rows_per_chunk = (rows + chunks - 1) / chunks;
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(chunks, 4), dim3(256), 0, s, ga);
    L_TRY(hipGetLastError());
    *chunks_out = chunks;
    *blocks_out = blocks;
    return SAFR_OK;
}

safr_status read_loss(safr_trainer* t, int blocks, hipStream_t s, double* loss) {
    std::vector<float> lp(blocks);
    L_TRY(hipMemcpyAsync(lp.data(), t->loss_part, blocks * sizeof(float), hipMemcpyDeviceToHost, s));
    L_TRY(hipStreamSynchronize(s));
    double acc = 0.0;
    for (float x : lp) acc += x;
    *loss = acc;
    return SAFR_OK;
}

}  // namespace

extern "C" {

safr_status safr_trainer_create(const safr_geometry* geo, int L, const double* heights, const double* weights,
                                const float* amp, int max_frames, safr_trainer** out, hipStream_t stream) {
    if (!out) return lfail(SAFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!geo || !heights || !weights || !amp || !geo->stars) return lfail(SAFR_ERR_ARG, "NULL argument");
    if (max_frames < 1) return lfail(SAFR_ERR_ARG, "max_frames must be >= 1");
    const int M = geo->M, J = geo->J;
    if (M != 32 && M != 64 && M != 128 && M != 256) return lfail(SAFR_ERR_UNSUPPORTED, "M = %d not supported", M);
    if (L < 1 || L > kMaxL || J < 1 || J > kMaxG) return lfail(SAFR_ERR_UNSUPPORTED, "J or L out of range");
    const int kind = geo->stars[0].kind;
    for (int g = 0; g < J; ++g)
        if (geo->stars[g].kind != kind) return lfail(SAFR_ERR_UNSUPPORTED, "training needs one kind of guide star");
    double wsum = 0.0;
    for (int l = 0; l < L; ++l) {
        if (!(weights[l] > 0.0)) return lfail(SAFR_ERR_GEOMETRY, "weights must be > 0");
        if (l > 0 && !(heights[l] > heights[l - 1])) return lfail(SAFR_ERR_GEOMETRY, "heights must ascend");
        wsum += weights[l];
    }
    if (kind == SAFR_LGS && !(heights[L - 1] < geo->h_lgs)) return lfail(SAFR_ERR_GEOMETRY, "layers above h_lgs");
    safr_trainer* t = new safr_trainer();
    t->M = M;
    t->G = J;
    t->L = L;
    t->r = std::min(J, L);
    t->Kh = M / 2 + 1;
    t->H = (size_t)t->Kh * M;
    t->stride = t->r * t->r + t->r + 1;
    t->max_frames = max_frames;
    const size_t H = t->H;
    const double T = M * geo->pitch / 2.0;
    double cl[kMaxL];
    for (int l = 0; l < L; ++l) cl[l] = kind == SAFR_LGS ? 1.0 - heights[l] / geo->h_lgs : 1.0;
    // FP64 SVD of A_n on the half spectrum (the precompute's kernel)
    double2 *W = nullptr, *Qd = nullptr;
    double* sig = nullptr;
    safr_status st = SAFR_OK;
    auto bail = [&](safr_status s2) {
        (void)hipFree(W);
        (void)hipFree(Qd);
        (void)hipFree(sig);
        free_trainer(t);
        return s2;
    };
#define T_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t _e = (expr);                                                                      \
        if (_e != hipSuccess) return bail(lfail(SAFR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e))); \
    } while (0)
    const int R = std::max(J, L), C = t->r;
    T_TRY(hipMalloc(&W, H * R * C * sizeof(double2)));
    T_TRY(hipMalloc(&Qd, H * C * C * sizeof(double2)));
    T_TRY(hipMalloc(&sig, H * C * sizeof(double)));
    PrecompArgs pa{};
    pa.M = M;
    pa.G = J;
    pa.L = L;
    pa.T = T;
    pa.beta = geo->beta;
    for (int g = 0; g < J; ++g) {
        pa.ax[g] = geo->stars[g].ax;
        pa.ay[g] = geo->stars[g].ay;
    }
    LearnSetupArgs sa{};
    for (int l = 0; l < L; ++l) {
        pa.h[l] = heights[l];
        pa.c[l] = cl[l];
        pa.gamma[l] = weights[l] / wsum;
        pa.sqrt_gamma[l] = std::sqrt(weights[l] / wsum);
        sa.c[l] = cl[l];
        sa.gamma[l] = pa.gamma[l];
        sa.sqrt_gamma[l] = pa.sqrt_gamma[l];
        for (int g = 0; g < J; ++g) {
            sa.sx[g * kMaxL + l] = geo->stars[g].ax * heights[l] / (cl[l] * geo->pitch);
            sa.sy[g * kMaxL + l] = geo->stars[g].ay * heights[l] / (cl[l] * geo->pitch);
        }
    }
    pa.W = W;
    pa.Q = Qd;
    pa.sigma = sig;
    T_TRY(launch_svd(pa, stream));
    LearnFreq& f = t->fq;
    T_TRY(hipMalloc(&f.U, H * J * C * sizeof(float2)));
    T_TRY(hipMalloc(&f.V, H * L * C * sizeof(float2)));
    T_TRY(hipMalloc(&f.inv_sigma, H * C * sizeof(float)));
    T_TRY(hipMalloc(&f.feat, H * C * 4 * sizeof(float)));
    T_TRY(hipMalloc(&f.s, H * L * sizeof(float)));
    T_TRY(hipMalloc(&f.ph, H * J * L * sizeof(float2)));
    T_TRY(hipMalloc(&f.mult, H * sizeof(float)));
    T_TRY(hipMalloc(&t->fq_dev, sizeof(LearnFreq)));
    T_TRY(hipMemcpy(t->fq_dev, &f, sizeof(LearnFreq), hipMemcpyHostToDevice));
    sa.M = M;
    sa.G = J;
    sa.L = L;
    sa.r = C;
    sa.T = T;
    sa.beta = geo->beta;
    sa.W = W;
    sa.Q = Qd;
    sa.sigma = sig;
    sa.freq = t->fq_dev;
    hipLaunchKernelGGL(learn_setup_kernel, dim3((unsigned)((H + 63) / 64)), dim3(64), 0, stream, sa);
    T_TRY(hipGetLastError());
    // amplitude, normalisation Z = sum_n w_n sum_l amp^2, noise scale sigma_n M = sqrt(Z) / M
    T_TRY(hipMalloc(&t->amp, H * L * sizeof(float)));
    T_TRY(hipMemcpy(t->amp, amp, H * L * sizeof(float), hipMemcpyHostToDevice));
    double Z = 0.0;
    for (int k = 0; k < t->Kh; ++k)
        for (int j = 0; j < M; ++j) {
            const bool nyq = (M % 2 == 0) && (j == M / 2 || k == M / 2);
            const double w = nyq ? 0.0 : (k == 0 ? 1.0 : 2.0);
            for (int l = 0; l < L; ++l) {
                const double a = amp[((size_t)l * t->Kh + k) * M + j];
                Z += w * a * a;
            }
        }
    t->Z = Z;
    t->noise_scale = (float)(std::sqrt(Z) / M);
    T_TRY(hipMalloc(&t->stats, (size_t)max_frames * H * t->stride * sizeof(float)));
    T_TRY(hipMalloc(&t->eta, (size_t)max_frames * sizeof(float)));
    T_TRY(hipMalloc(&t->params, 8705 * sizeof(float)));
    T_TRY(hipMalloc(&t->m, 8705 * sizeof(float)));
    T_TRY(hipMalloc(&t->v, 8705 * sizeof(float)));
    T_TRY(hipMalloc(&t->grad, 8705 * sizeof(float)));
    T_TRY(hipMemsetAsync(t->params, 0, 8705 * sizeof(float), stream));
    T_TRY(hipMemsetAsync(t->m, 0, 8705 * sizeof(float), stream));
    T_TRY(hipMemsetAsync(t->v, 0, 8705 * sizeof(float), stream));
    T_TRY(hipStreamSynchronize(stream));
#undef T_TRY
    (void)hipFree(W);
    (void)hipFree(Qd);
    (void)hipFree(sig);
    (void)st;
    *out = t;
    return SAFR_OK;
}

safr_status safr_trainer_add_frames(safr_trainer* t, int count, const void* zl, const void* zn, const float* eta,
                                    hipStream_t s) {
    if (!t || !zl || !zn || !eta || count < 1) return lfail(SAFR_ERR_ARG, "bad argument");
    if (t->nframes + count > t->max_frames) return lfail(SAFR_ERR_STATE, "trainer holds at most %d frames", t->max_frames);
    for (int i = 0; i < count; ++i)
        if (!(eta[i] > 0.f)) return lfail(SAFR_ERR_ARG, "noise levels must be > 0");
    L_TRY(hipMemcpy(t->eta + t->nframes, eta, count * sizeof(float), hipMemcpyHostToDevice));
    LearnStatsArgs a{};
    a.freq = t->fq_dev;
    a.amp = t->amp;
    a.zl = reinterpret_cast<const float2*>(zl);
    a.zn = reinterpret_cast<const float2*>(zn);
    a.eta = t->eta + t->nframes;
    a.stats = t->stats;
    a.noise_scale = t->noise_scale;
    a.G = t->G;
    a.L = t->L;
    a.r = t->r;
    a.count = count;
    a.first = t->nframes;
    a.stride = t->stride;
    a.H = t->H;
    const size_t n = (size_t)count * t->H;
    hipLaunchKernelGGL(learn_stats_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a);
    L_TRY(hipGetLastError());
    t->nframes += count;
    return SAFR_OK;
}

safr_status safr_trainer_set_params(safr_trainer* t, const float* host) {
    if (!t || !host) return lfail(SAFR_ERR_ARG, "NULL argument");
    L_TRY(hipMemcpy(t->params, host, 8705 * sizeof(float), hipMemcpyHostToDevice));
    L_TRY(hipMemset(t->m, 0, 8705 * sizeof(float)));
    L_TRY(hipMemset(t->v, 0, 8705 * sizeof(float)));
    t->step = 0;
    return SAFR_OK;
}

safr_status safr_trainer_get_params(const safr_trainer* t, float* host) {
    if (!t || !host) return lfail(SAFR_ERR_ARG, "NULL argument");
    L_TRY(hipMemcpy(host, t->params, 8705 * sizeof(float), hipMemcpyDeviceToHost));
    return SAFR_OK;
}

safr_status safr_trainer_get_state(const safr_trainer* t, float* m, float* v, int* step) {
    if (!t || !m || !v || !step) return lfail(SAFR_ERR_ARG, "NULL argument");
    L_TRY(hipMemcpy(m, t->m, 8705 * sizeof(float), hipMemcpyDeviceToHost));
    L_TRY(hipMemcpy(v, t->v, 8705 * sizeof(float), hipMemcpyDeviceToHost));
    *step = t->step;
    return SAFR_OK;
}

safr_status safr_trainer_set_state(safr_trainer* t, const float* m, const float* v, int step) {
    if (!t || !m || !v) return lfail(SAFR_ERR_ARG, "NULL argument");
    if (step < 0) return lfail(SAFR_ERR_ARG, "step must be >= 0");
    for (int i = 0; i < 8705; ++i)
        if (!std::isfinite(m[i]) || !std::isfinite(v[i]) || v[i] < 0.f)
            return lfail(SAFR_ERR_ARG, "Adam moments must be finite (second moments >= 0)");
    L_TRY(hipMemcpy(t->m, m, 8705 * sizeof(float), hipMemcpyHostToDevice));
    L_TRY(hipMemcpy(t->v, v, 8705 * sizeof(float), hipMemcpyHostToDevice));
    t->step = step;
    return SAFR_OK;
}

safr_status safr_trainer_gradient(safr_trainer* t, int nb, const int* frames, float* grad, double* loss,
                                  hipStream_t s) {
    if (!t || !frames || nb < 1) return lfail(SAFR_ERR_ARG, "bad argument");
    int chunks = 0, blocks = 0;
    safr_status st = run_batch(t, nb, frames, s, &chunks, &blocks);
    if (st != SAFR_OK) return st;
    MlpAdamArgs aa{};
    aa.partials = t->partials;
    aa.chunks = chunks;
    aa.grad_out = t->grad;
    aa.update = 0;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((8705 + 255) / 256), dim3(256), 0, s, aa);
    L_TRY(hipGetLastError());
    if (grad) {
        L_TRY(hipMemcpyAsync(grad, t->grad, 8705 * sizeof(float), hipMemcpyDeviceToHost, s));
        L_TRY(hipStreamSynchronize(s));
    }
    if (loss) return read_loss(t, blocks, s, loss);
    return SAFR_OK;
}

safr_status safr_trainer_step(safr_trainer* t, int nb, const int* frames, float lr, double* loss, hipStream_t s) {
    if (!t || !frames || nb < 1 || !(lr > 0.f)) return lfail(SAFR_ERR_ARG, "bad argument");
    int chunks = 0, blocks = 0;
    safr_status st = run_batch(t, nb, frames, s, &chunks, &blocks);
    if (st != SAFR_OK) return st;
    t->step += 1;
    MlpAdamArgs aa{};
    aa.partials = t->partials;
    aa.chunks = chunks;
    aa.grad_out = nullptr;
    aa.update = 1;
    aa.params = t->params;
    aa.m = t->m;
    aa.v = t->v;
    aa.lr = lr;
    aa.b1 = 0.9f;
    aa.b2 = 0.999f;
    aa.eps = 1e-8f;
    aa.b1t = (float)std::pow(0.9, t->step);
    aa.b2t = (float)std::pow(0.999, t->step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((8705 + 255) / 256), dim3(256), 0, s, aa);
    L_TRY(hipGetLastError());
    if (loss) return read_loss(t, blocks, s, loss);
    return SAFR_OK;
}

namespace {

// the training objective of the listed frames for the optimal (mode 0) or Tikhonov (mode 1) filter factors
safr_status filter_eval(safr_trainer* t, int nb, const int* frames, int mode, double alpha, float* phi_host,
                        double* loss, hipStream_t s) {
    if (!t || !frames || nb < 1 || !loss) return lfail(SAFR_ERR_ARG, "bad argument");
    for (int i = 0; i < nb; ++i)
        if (frames[i] < 0 || frames[i] >= t->nframes) return lfail(SAFR_ERR_ARG, "frame index %d out of range", frames[i]);
    int* dframes = nullptr;
    double* dloss = nullptr;
    float* dphi = nullptr;
    hipError_t e = hipMalloc(&dframes, nb * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&dloss, t->H * sizeof(double));
    if (e == hipSuccess && phi_host) e = hipMalloc(&dphi, t->H * t->r * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(dframes, frames, nb * sizeof(int), hipMemcpyHostToDevice);
    std::vector<double> lh(t->H);
    if (e == hipSuccess) {
        FilterEvalArgs a{};
        a.freq = t->fq_dev;
        a.stats = t->stats;
        a.frames = dframes;
        a.phi = dphi;
        a.loss = dloss;
        a.alpha = alpha;
        a.nb = nb;
        a.r = t->r;
        a.stride = t->stride;
        a.mode = mode;
        a.H = t->H;
        hipLaunchKernelGGL(filter_eval_kernel, dim3((unsigned)((t->H + 63) / 64)), dim3(64), 0, s, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(lh.data(), dloss, t->H * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && phi_host) e = hipMemcpyAsync(phi_host, dphi, t->H * t->r * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dframes);
    (void)hipFree(dloss);
    (void)hipFree(dphi);
    if (e != hipSuccess) return lfail(SAFR_ERR_DEVICE, "filter evaluation failed: %s", hipGetErrorString(e));
    double acc = 0.0;
    for (double x : lh) acc += x;
    *loss = acc / (t->Z * nb);
    return SAFR_OK;
}

}  // namespace

safr_status safr_trainer_optimal_filter(safr_trainer* t, int nb, const int* frames, float* phi, double* loss,
                                        hipStream_t s) {
    return filter_eval(t, nb, frames, 0, 0.0, phi, loss, s);
}

safr_status safr_trainer_tikhonov_loss(safr_trainer* t, int nb, const int* frames, double alpha, double* loss,
                                       hipStream_t s) {
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return lfail(SAFR_ERR_ARG, "alpha must be >= 0");
    return filter_eval(t, nb, frames, 1, alpha, nullptr, loss, s);
}

int safr_trainer_frames(const safr_trainer* t) { return t ? t->nframes : 0; }

void safr_trainer_destroy(safr_trainer* t) { free_trainer(t); }

safr_status safr_mlp_infer(const float* params, const float* feats, int rows, double noise, float* phi,
                           hipStream_t s) {
    if (!params || !feats || !phi || rows < 0 || !(noise > 0.0)) return lfail(SAFR_ERR_ARG, "bad argument");
    if (rows == 0) return SAFR_OK;
    float* p = nullptr;
    L_TRY(hipMalloc(&p, 8705 * sizeof(float)));
    hipError_t e = hipMemcpy(p, params, 8705 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_infer(p, feats, phi, rows, (float)std::log10(noise), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(p);
    if (e != hipSuccess) return lfail(SAFR_ERR_DEVICE, "network inference failed: %s", hipGetErrorString(e));
    return SAFR_OK;
}

}  // extern "C"
