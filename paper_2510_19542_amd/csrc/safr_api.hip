// Host side of the SAFR C ABI: validation of the geometry (Sec. 2), the
// soft-real-time precomputation (Alg. 2) driven on the GPU, and the dispatch of
// the hard-real-time kernels (Alg. 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "safr_internal.h"

using namespace safr;

namespace {

thread_local std::string g_last_error = "no error";

safr_status fail(safr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(SAFR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));  \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool supported_M(int M) { return M == 32 || M == 64 || M == 128 || M == 256; }

int team_size(int M) { return M == 256 ? 16 : (M == 32 ? 4 : 8); }

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

namespace safr {
safr_status set_error(safr_status st, const char* msg) {
    g_last_error = msg;
    return st;
}
}  // namespace safr

struct safr_plan {
    int n = 0, M = 0, J = 0, L = 0, Kh = 0;
    int ngroups = 0, mixed = 0;
    double pitch = 0.0, T = 0.0;
    int gsize[2] = {0, 0}, gkind[2] = {0, 0};
    int gstar[2][kMaxG] = {};
    double galpha[2] = {0.0, 0.0};
    double c_out[kMaxL] = {};
    double heights[kMaxL] = {};
    size_t bcount[2] = {0, 0};      // complex entries per group (FP64 export layout)
    size_t boff[2] = {0, 0};        // group offsets in B64
    size_t boff32[2] = {0, 0};      // group offsets in B32 (column-block layout, zero padded)
    float tt_b[3] = {0, 0, 0}, tt_c[3] = {0, 0, 0};
    int p0 = 0;
    // device memory owned by the plan
    double2* B64 = nullptr;
    float2* B32 = nullptr;
    uint16_t* Apack = nullptr;
    float2* Bm = nullptr;           // group 0's B in the matrix-core lane layout (FP32 column pass, 4 frames)
    size_t apack_off[2] = {0, 0};
    int mf_lt[2] = {0, 0}, mf_ntile[2] = {0, 0}, mf_ppm[2] = {0, 0};
    float2* tw = nullptr;
    float2* Xh = nullptr;           // DFT2 of x * pupil (tip/tilt plane transforms), [Kh][M]
    float2* Yh = nullptr;
    float* P = nullptr;             // natural-star basis images [L][nb][M][M] (mixed asterisms)
    int nb = 0;
    // kept for refreshes of the filter (safr_update_alpha): per group the geometry of A_n and its SVD
    // (W, Q, sigma owned by the plan), the FP64 transforms of x * pupil and y * pupil, the filter in use
    PrecompArgs pre[2] = {};
    double2* X64 = nullptr;
    double2* Y64 = nullptr;
    int filter = SAFR_FILTER_TIKHONOV;
    int weighted = 0;               // B was made with a per-frequency alpha map
    int imported = 0;               // B replaced by safr_import_B (the kept SVDs no longer describe it)
    unsigned char* pupil = nullptr;
    int tt_mode[kMaxJ] = {};        // per star: 0 none, 1 remove tip/tilt, 2 plane only
    float4* polc_tab = nullptr;     // [J][L] line-of-sight sampling of the output grids (closed loop)
    float* strehl_part = nullptr;   // per-chunk moments of the Strehl estimate (grown on demand)
    size_t strehl_part_floats = 0;
    void* ws_own = nullptr;
    size_t ws_own_bytes = 0;
    void* ws_user = nullptr;
    size_t ws_user_bytes = 0;
    // tuning
    int row_teams = 0, out_rows = 0, out_frames = 1, mfma_frames = 16, col_frames = 1, col_nf = 1, col_prefetch = 1;
    int col_mfma = 0;               // FP32 column pass with 4 frames: the apply on the matrix cores
    int col_frames_auto = 1;        // column frames per block chosen per launch (until set or autotuned)
    int seq_frames = 0;             // frames per launch sequence (0: from kSequenceBytes), see SAFR_OPT_SEQ_FRAMES
    int fused = 1;                  // one-kernel step where the shape has one, see SAFR_OPT_FUSED
    int use_graph = 0;
    int deadline_us = 0;            // loop-step deadline (0: off), see SAFR_OPT_DEADLINE_US
    unsigned long long deadline_ticks = 0;
    unsigned long long* dstats = nullptr;   // device: steps, misses, last, max (wall-clock ticks), start stamp
    double ticks_per_us = 0.0;
    int check_finite = 0;           // debug: scan inputs for non-finite values first (synchronises)
    int* dfirst = nullptr;          // first non-finite frame found by the check
    // graph cache
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_frames = 0, g_prec = 0;
    const float* g_wf = nullptr;
    float* g_out = nullptr;
    hipStream_t g_stream = nullptr;
    // graph cache of the closed-loop step
    hipGraphExec_t lexec = nullptr;
    hipGraph_t lgraph = nullptr;
    int l_frames = 0;
    float l_gain = 0.f;
    const float* l_wf = nullptr;
    const float* l_ain = nullptr;
    float* l_aout = nullptr;
    hipStream_t l_stream = nullptr;
};

namespace {

// frames of one call: the row pass's grid has one z index per frame
constexpr int kMaxFrames = 65535;

// workspace: row spectra R, layer column spectra C, plane parts of the row chunks (sized for the smallest row blocks)
size_t ws_r(const safr_plan* p, int frames) { return align256((size_t)frames * p->J * p->Kh * p->n * sizeof(float2)); }
size_t ws_c(const safr_plan* p, int frames) {
    return align256((size_t)frames * p->L * p->Kh * p->M * sizeof(float2));
}
// (the plane coefficients of every row chunk, then, for more than kPlaneLanes chunks, their sums)
size_t ws_mom(const safr_plan* p, int frames) {
    return align256((size_t)frames * p->J * ((p->n + 1) / 2) * sizeof(float2));
}
size_t ws_m(const safr_plan* p, int frames) {
    return ws_mom(p, frames) + align256((size_t)frames * p->J * sizeof(float2));
}
// pseudo-open-loop wavefronts of the closed-loop step
size_t ws_w(const safr_plan* p, int frames) { return align256((size_t)frames * p->J * p->n * p->n * sizeof(float)); }
// A call with more frames runs as several launch sequences (row, column and output pass) of about equal size,
// each with at most this many bytes of intermediate spectra (R and C), so that they stay in the 256 MB
// Infinity Cache next to B and the basis images: 69 MORFEO-like frames (3.0 MB each; measured: 128 frames as
// one sequence 304 us, as two of 64 243 us).
constexpr size_t kSequenceBytes = size_t(200) << 20;
int sequence_frames(const safr_plan* p) {
    if (p->seq_frames > 0) return p->seq_frames;
    const size_t per = (size_t)p->J * p->Kh * p->n * sizeof(float2) + (size_t)p->L * p->Kh * p->M * sizeof(float2);
    return (int)std::max<size_t>(1, std::min<size_t>(kSequenceBytes / per, kMaxFrames));
}

// Workspace of a call: R, C and the plane parts of its largest launch sequence (each sequence starts at the
// beginning of the workspace), then the pseudo-open-loop wavefronts of all its frames (closed-loop step).
size_t ws_seq(const safr_plan* p, int frames) {
    const int f = std::min(frames, sequence_frames(p));
    return ws_r(p, f) + ws_c(p, f) + ws_m(p, f);
}
size_t ws_bytes(const safr_plan* p, int frames) { return ws_seq(p, frames) + ws_w(p, frames); }


// captured graphs hold launch shapes and pointers: dropped whenever a tuning option changes
void drop_graphs(safr_plan* p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->lexec) (void)hipGraphExecDestroy(p->lexec);
    if (p->lgraph) (void)hipGraphDestroy(p->lgraph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->lexec = nullptr;
    p->lgraph = nullptr;
}

void free_plan(safr_plan* p) {
    if (!p) return;
    drop_graphs(p);
    (void)hipFree(p->B64);
    (void)hipFree(p->B32);
    (void)hipFree(p->Apack);
    (void)hipFree(p->Bm);
    (void)hipFree(p->tw);
    (void)hipFree(p->Xh);
    (void)hipFree(p->Yh);
    (void)hipFree(p->P);
    (void)hipFree(p->pupil);
    (void)hipFree(p->polc_tab);
    (void)hipFree(p->strehl_part);
    for (int gi = 0; gi < 2; ++gi) {
        (void)hipFree(p->pre[gi].W);
        (void)hipFree(p->pre[gi].Q);
        (void)hipFree(p->pre[gi].sigma);
    }
    (void)hipFree(p->X64);
    (void)hipFree(p->Y64);
    (void)hipFree(p->dfirst);
    (void)hipFree(p->dstats);
    (void)hipFree(p->ws_own);
    delete p;
}

// Inverse of the 3 x 3 normal matrix of the least-squares fit of [1, x, y] over the pupil.
bool tt_inverse(const std::vector<unsigned char>& pup, int n, double inv[9]) {
    double N[9] = {0};
    const double half = 0.5 * (n - 1);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (!pup[(size_t)i * n + j]) continue;
            const double v[3] = {1.0, i - half, j - half};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) N[3 * a + b] += v[a] * v[b];
        }
    const double det = N[0] * (N[4] * N[8] - N[5] * N[7]) - N[1] * (N[3] * N[8] - N[5] * N[6]) +
                       N[2] * (N[3] * N[7] - N[4] * N[6]);
    if (!(std::fabs(det) > 1e-12)) return false;
    inv[0] = (N[4] * N[8] - N[5] * N[7]) / det;
    inv[1] = (N[2] * N[7] - N[1] * N[8]) / det;
    inv[2] = (N[1] * N[5] - N[2] * N[4]) / det;
    inv[3] = (N[5] * N[6] - N[3] * N[8]) / det;
    inv[4] = (N[0] * N[8] - N[2] * N[6]) / det;
    inv[5] = (N[2] * N[3] - N[0] * N[5]) / det;
    inv[6] = (N[3] * N[7] - N[4] * N[6]) / det;
    inv[7] = (N[1] * N[6] - N[0] * N[7]) / det;
    inv[8] = (N[0] * N[4] - N[1] * N[3]) / det;
    return true;
}

// DFT2 (FP64, direct) of x * pupil and y * pupil zero-extended at offset p0, half spectrum [k][j].
void tt_transforms(const std::vector<unsigned char>& pup, int n, int M, int p0, std::vector<double2>& X,
                   std::vector<double2>& Y) {
    const int Kh = M / 2 + 1;
    const double half = 0.5 * (n - 1);
    // exp(-2 pi i e / M) for e = 0..M-1, indexed by the exponent reduced mod M
    std::vector<std::pair<double, double>> tw(M);
    for (int e = 0; e < M; ++e) {
        const double ang = -2.0 * M_PI * (double)e / M;
        tw[e] = std::make_pair(std::cos(ang), std::sin(ang));
    }
    auto w = [M, &tw](long e) { return tw[e % M]; };
    // row sums at each k: rx = sum_q mask e^{-2 pi i k (p0+q)/M}, ry = sum_q (q - half) mask e^{...}
    std::vector<double> rxr((size_t)n * Kh), rxi((size_t)n * Kh), ryr((size_t)n * Kh), ryi((size_t)n * Kh);
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < Kh; ++k) {
            double ar = 0, ai = 0, br = 0, bi = 0;
            for (int q = 0; q < n; ++q) {
                if (!pup[(size_t)p * n + q]) continue;
                const auto e = w((long)k * (p0 + q));
                ar += e.first;
                ai += e.second;
                br += (q - half) * e.first;
                bi += (q - half) * e.second;
            }
            rxr[(size_t)p * Kh + k] = ar;
            rxi[(size_t)p * Kh + k] = ai;
            ryr[(size_t)p * Kh + k] = br;
            ryi[(size_t)p * Kh + k] = bi;
        }
    X.assign((size_t)Kh * M, make_double2(0.0, 0.0));
    Y.assign((size_t)Kh * M, make_double2(0.0, 0.0));
    for (int k = 0; k < Kh; ++k)
        for (int j = 0; j < M; ++j) {
            double xr = 0, xi = 0, yr = 0, yi = 0;
            for (int p = 0; p < n; ++p) {
                const auto e = w((long)j * (p0 + p));
                const double cr = rxr[(size_t)p * Kh + k], ci = rxi[(size_t)p * Kh + k];
                const double dr = ryr[(size_t)p * Kh + k], di = ryi[(size_t)p * Kh + k];
                const double x = p - half;
                xr += x * (e.first * cr - e.second * ci);
                xi += x * (e.first * ci + e.second * cr);
                yr += e.first * dr - e.second * di;
                yi += e.first * di + e.second * dr;
            }
            X[(size_t)k * M + j] = make_double2(xr, xi);
            Y[(size_t)k * M + j] = make_double2(yr, yi);
        }
}

// stage >= 0: only that stage's launches (0 row pass, 1 column pass, 2 output pass), on the inputs an earlier
// full sequence left in the workspace
safr_status launch_all(safr_plan* p, int frames, const float* wf, float* out, int precision,
                       void* ws, hipStream_t s, hipEvent_t* ev = nullptr, const float* prev = nullptr,
                       float gain = 1.f, int stage = -1);

// per-frequency alpha multipliers: finite, >= 0 and point-symmetric (B must stay Hermitian)
safr_status check_alpha_weight(int M, const double* w) {
    for (int j = 0; j < M; ++j)
        for (int k = 0; k < M; ++k) {
            const double v = w[(size_t)j * M + k];
            if (!(v >= 0.0) || !std::isfinite(v))
                return fail(SAFR_ERR_ARG, "alpha_weight[%d][%d] must be finite and >= 0", j, k);
            if (v != w[(size_t)((M - j) % M) * M + (M - k) % M])
                return fail(SAFR_ERR_ARG, "alpha_weight must be point-symmetric (w[j][k] = w[-j][-k])");
        }
    return SAFR_OK;
}

#define BT_TRY(expr)                                                                                \
    {                                                                                               \
        hipError_t _e = (expr);                                                                     \
        if (_e != hipSuccess) {                                                                     \
            st = fail(SAFR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));            \
            break;                                                                                  \
        }                                                                                           \
    }

// natural-star basis images of a mixed asterism from the natural group's FP64 B (the natural stars enter
// the output pass through them); synchronises `s`
safr_status build_basis(safr_plan* p, hipStream_t s) {
    const int M = p->M, L = p->L, Gn = p->gsize[1];
    p->nb = 2 * Gn;
    safr_status st = SAFR_OK;
    double2* tw64 = nullptr;
    double2* Tb = nullptr;
    double* Eb = nullptr;
    do {
        std::vector<double2> t64(M);
        for (int e = 0; e < M; ++e) t64[e] = make_double2(std::cos(2.0 * M_PI * e / M), std::sin(2.0 * M_PI * e / M));
        BT_TRY(hipMalloc(&tw64, M * sizeof(double2)));
        BT_TRY(hipMemcpy(tw64, t64.data(), M * sizeof(double2), hipMemcpyHostToDevice));
        BT_TRY(hipMalloc(&Tb, (size_t)L * p->nb * p->Kh * M * sizeof(double2)));
        BT_TRY(hipMalloc(&Eb, (size_t)L * p->nb * M * M * sizeof(double)));
        if (!p->P) BT_TRY(hipMalloc(&p->P, (size_t)L * p->nb * M * M * sizeof(float)));
        BasisArgs ba{};
        ba.M = M;
        ba.L = L;
        ba.G = Gn;
        for (int l = 0; l < L; ++l) ba.c[l] = p->c_out[l];
        ba.B64 = p->B64 + p->boff[1];
        ba.X = p->X64;
        ba.Y = p->Y64;
        ba.tw64 = tw64;
        ba.T = Tb;
        ba.E = Eb;
        ba.P = p->P;
        BT_TRY(launch_ngs_basis(ba, s));
        BT_TRY(hipStreamSynchronize(s));
    } while (0);
    (void)hipFree(tw64);
    (void)hipFree(Tb);
    (void)hipFree(Eb);
    return st;
}

// BF16 hi/lo tiles of the real-split B for the matrix-core apply (M <= 128), column group only; and (any M)
// the FP32 B in the lane layout of the four-frame column pass's matrix-core apply
safr_status build_mfma_b(safr_plan* p, hipStream_t s) {
    const int M = p->M, L = p->L, G = p->gsize[0];
    if (!p->col_mfma || !cols_fixed_shape(M, L, G, p->mixed ? 1 : 0)) return SAFR_OK;
    if (!p->Bm) HIP_TRY(hipMalloc(&p->Bm, mfma_b_count(M, L, G) * sizeof(float2)));
    HIP_TRY(launch_pack_mfma_b(M, L, G, p->B32 + p->boff32[0], p->Bm, s));
    return SAFR_OK;
}

safr_status build_pack(safr_plan* p, hipStream_t s) {
    const int M = p->M, L = p->L, G = p->gsize[0];
    {
        const safr_status st = build_mfma_b(p, s);
        if (st != SAFR_OK) return st;
    }
    if (M > 128) return SAFR_OK;
    int nf = 0;
    for (int cand : {16, 8, 4})
        if (!nf && mfma_lds_bytes(M, cand, G, L) <= 160 * 1024) nf = cand;
    if (!nf) return SAFR_OK;
    safr_status st = SAFR_OK;
    do {
        if (!p->Apack) p->mfma_frames = nf;
        const int lt = std::min(L, 8), ntile = (L + lt - 1) / lt;
        int ppm = std::max(1, std::min(16 / (2 * lt), 32 / (2 * G)));
        while (ppm & (ppm - 1)) --ppm;                 // a power of two, so it divides M
        p->mf_lt[0] = lt;
        p->mf_ntile[0] = ntile;
        p->mf_ppm[0] = ppm;
        const size_t tot = (size_t)p->Kh * (M / ppm) * ntile * 2 * 64 * 8;
        if (!p->Apack) BT_TRY(hipMalloc(&p->Apack, tot * sizeof(uint16_t)));
        BT_TRY(launch_pack_bf16(M, L, G, p->B32 + p->boff32[0], p->Apack, lt, ntile, ppm, s));
    } while (0);
    return st;
}


PolcArgs polc_args(const safr_plan* p, const float* wf, const float* layers, float weight, float* out) {
    PolcArgs a{};
    a.wf = wf;
    a.layers = layers;
    a.out = out;
    a.pupil = p->pupil;
    a.tab = p->polc_tab;
    a.weight = weight;
    a.n = p->n;
    a.M = p->M;
    a.J = p->J;
    a.L = p->L;
    return a;
}

// Debug input check (SAFR_OPT_CHECK_FINITE): wavefronts at pupil pixels and, when given, layer-shaped
// inputs everywhere; synchronises the stream and names the first frame with a non-finite value.
safr_status check_inputs(safr_plan* p, int frames, const float* wf, const float* layers, hipStream_t s) {
    const int none = INT_MAX;
    HIP_TRY(hipMemcpyAsync(p->dfirst, &none, sizeof(int), hipMemcpyHostToDevice, s));
    const int pix = p->n * p->n;
    HIP_TRY(launch_finite_check(wf, p->pupil, pix, p->J * pix, frames, p->dfirst, s));
    if (layers) HIP_TRY(launch_finite_check(layers, nullptr, 1, p->L * p->M * p->M, frames, p->dfirst, s));
    int first = none;
    HIP_TRY(hipMemcpyAsync(&first, p->dfirst, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (first != none) return fail(SAFR_ERR_NUMERIC, "non-finite input in frame %d", first);
    return SAFR_OK;
}

// Alg. 3 without its wavefront reconstruction: POLC into the workspace, the reconstruction with
// the integrator fused into the output pass
safr_status launch_loop(safr_plan* p, int frames, const float* wf, const float* a_in, float gain, float* a_out,
                        void* ws, hipStream_t s) {
    float* psi = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + ws_seq(p, frames));
    if (p->deadline_ticks) HIP_TRY(launch_deadline_start(p->dstats, s));
    HIP_TRY(launch_polc(polc_args(p, wf, a_in, 1.f, psi), frames, s));
    const safr_status st = launch_all(p, frames, psi, a_out, SAFR_FP32, ws, s, nullptr, a_in, gain);
    if (st != SAFR_OK) return st;
    if (p->deadline_ticks) HIP_TRY(launch_deadline_end(p->dstats, p->deadline_ticks, s));
    return SAFR_OK;
}

}  // namespace

extern "C" {

const char* safr_last_error(void) { return g_last_error.c_str(); }

safr_status safr_precompute(const safr_geometry* geo, int L, const double* heights, const double* weights,
                            double alpha, safr_plan** out, hipStream_t stream) {
    if (!out) return fail(SAFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!geo || !heights || !weights) return fail(SAFR_ERR_ARG, "geometry, heights or weights is NULL");
    if (!geo->stars || geo->J < 1) return fail(SAFR_ERR_ARG, "need J >= 1 stars");
    if (L < 1) return fail(SAFR_ERR_ARG, "need L >= 1 layers");
    if (L > kMaxL) return fail(SAFR_ERR_UNSUPPORTED, "L = %d exceeds %d", L, kMaxL);
    const int M = geo->M, n = geo->n, J = geo->J;
    if (!supported_M(M)) return fail(SAFR_ERR_UNSUPPORTED, "M = %d not in {32, 64, 128, 256}", M);
    if (n < 1) return fail(SAFR_ERR_ARG, "n = %d < 1", n);
    if (n > M) return fail(SAFR_ERR_UNSUPPORTED, "n = %d exceeds M = %d", n, M);
    if (!(geo->pitch > 0.0) || !std::isfinite(geo->pitch)) return fail(SAFR_ERR_ARG, "pitch must be > 0");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SAFR_ERR_ARG, "alpha must be >= 0");
    if (!(geo->beta >= 0.0) || !std::isfinite(geo->beta)) return fail(SAFR_ERR_ARG, "beta must be >= 0");
    if (!(geo->alpha_tt >= 0.0) || !std::isfinite(geo->alpha_tt))
        return fail(SAFR_ERR_ARG, "alpha_tt must be >= 0");
    if (geo->filter != SAFR_FILTER_TIKHONOV && geo->filter != SAFR_FILTER_MLP && geo->filter != SAFR_FILTER_TSVD)
        return fail(SAFR_ERR_ARG, "unknown filter %d", geo->filter);
    if (geo->alpha_weight) {
        if (geo->filter == SAFR_FILTER_MLP) return fail(SAFR_ERR_ARG, "alpha_weight needs the Tikhonov or TSVD filter");
        const safr_status ws = check_alpha_weight(M, geo->alpha_weight);
        if (ws != SAFR_OK) return ws;
    }
    if (geo->filter == SAFR_FILTER_MLP && (!geo->mlp || !(geo->noise > 0.0)))
        return fail(SAFR_ERR_ARG, "learned filter needs parameters and noise > 0");
    int nl = 0, nn = 0;
    for (int g = 0; g < J; ++g) {
        const safr_star& st = geo->stars[g];
        if (st.kind != SAFR_NGS && st.kind != SAFR_LGS) return fail(SAFR_ERR_ARG, "star %d: bad kind", g);
        if (!std::isfinite(st.ax) || !std::isfinite(st.ay)) return fail(SAFR_ERR_ARG, "star %d: bad angle", g);
        (st.kind == SAFR_LGS ? nl : nn)++;
    }
    double wsum = 0.0;
    for (int l = 0; l < L; ++l) {
        if (!std::isfinite(heights[l]) || heights[l] < 0.0)
            return fail(SAFR_ERR_GEOMETRY, "height %d must be finite and >= 0", l);
        if (l > 0 && !(heights[l] > heights[l - 1]))
            return fail(SAFR_ERR_GEOMETRY, "heights must be strictly ascending");
        if (!(weights[l] > 0.0) || !std::isfinite(weights[l]))
            return fail(SAFR_ERR_GEOMETRY, "weight %d must be > 0", l);
        wsum += weights[l];
    }
    if (nl > 0) {
        if (!(geo->h_lgs > 0.0)) return fail(SAFR_ERR_GEOMETRY, "h_lgs must be > 0 with laser stars");
        if (!(heights[L - 1] < geo->h_lgs)) return fail(SAFR_ERR_GEOMETRY, "layers must lie below h_lgs");
    }
    if (nl > kMaxG || nn > kMaxG) return fail(SAFR_ERR_UNSUPPORTED, "more than %d stars of one kind", kMaxG);

    safr_plan* p = new safr_plan();
    p->n = n;
    p->M = M;
    p->J = J;
    p->L = L;
    p->Kh = M / 2 + 1;
    p->pitch = geo->pitch;
    p->T = M * geo->pitch / 2.0;
    p->p0 = (M - n + 1) / 2;
    p->mixed = (nl > 0 && nn > 0);
    // groups: mixed -> 0 = laser stars (alpha), 1 = natural stars (alpha_tt)
    if (p->mixed) {
        p->ngroups = 2;
        p->gkind[0] = SAFR_LGS;
        p->gkind[1] = SAFR_NGS;
        p->galpha[0] = alpha;
        p->galpha[1] = geo->alpha_tt;
    } else {
        p->ngroups = 1;
        p->gkind[0] = nl > 0 ? SAFR_LGS : SAFR_NGS;
        p->galpha[0] = alpha;
    }
    for (int g = 0; g < J; ++g) {
        const int gi = p->mixed ? (geo->stars[g].kind == SAFR_LGS ? 0 : 1) : 0;
        p->gstar[gi][p->gsize[gi]++] = g;
    }
    double cgrp[2][kMaxL];
    for (int gi = 0; gi < p->ngroups; ++gi)
        for (int l = 0; l < L; ++l)
            cgrp[gi][l] = p->gkind[gi] == SAFR_LGS ? 1.0 - heights[l] / geo->h_lgs : 1.0;
    for (int l = 0; l < L; ++l) {
        p->c_out[l] = cgrp[0][l];
        p->heights[l] = heights[l];
    }

    // domain condition c_l Omega_A + alpha_g h_l in c_l Omega_T (Sec. 2); skipped when the
    // data covers the whole periodic grid (n == M)
    if (n < M) {
        const double half = 0.5 * (n - 1) * geo->pitch;
        for (int gi = 0; gi < p->ngroups; ++gi)
            for (int l = 0; l < L; ++l)
                for (int m = 0; m < p->gsize[gi]; ++m) {
                    const safr_star& st = geo->stars[p->gstar[gi][m]];
                    const double c = cgrp[gi][l];
                    const double ext = c * half + std::max(std::fabs(st.ax), std::fabs(st.ay)) * heights[l];
                    if (ext > c * p->T * (1.0 + 1e-12)) {
                        free_plan(p);
                        return fail(SAFR_ERR_DOMAIN, "star %d at layer %d leaves the periodic domain",
                                    p->gstar[gi][m], l);
                    }
                }
    }

    std::vector<unsigned char> pup((size_t)n * n, 1);
    if (geo->pupil)
        for (size_t i = 0; i < pup.size(); ++i) pup[i] = geo->pupil[i] ? 1 : 0;
    std::vector<int> mode(J, 0);
    if (p->mixed) {
        double inv[9];
        if (!tt_inverse(pup, n, inv)) {
            free_plan(p);
            return fail(SAFR_ERR_GEOMETRY, "pupil too small for a tip/tilt fit");
        }
        for (int a = 0; a < 3; ++a) {
            p->tt_b[a] = (float)inv[3 + a];
            p->tt_c[a] = (float)inv[6 + a];
        }
        for (int g = 0; g < J; ++g) mode[g] = geo->stars[g].kind == SAFR_LGS ? 1 : 2;
    }

    // tuning defaults
    const int T = team_size(M);
    p->row_teams = std::min(256 / T, std::max(1, (n + 1) / 2));
    if (M == 256) p->row_teams = std::min(p->row_teams, 8);
    p->out_rows = M >= 128 ? 8 : (M == 64 ? 16 : 32);
    p->out_frames = out_frames_per_iter(M, p->out_rows);
    p->col_nf = M == 256 ? 4 : 2;           // 4 frames at once spill registers at M = 128
    p->col_frames = p->col_nf;

    safr_status st = SAFR_OK;
    float* feats = nullptr;
    float* phi = nullptr;
    float* mlp_dev = nullptr;
    double* aw_dev = nullptr;
    int* dbad = nullptr;
    do {
        size_t total = 0, total32 = 0;
        const int cpw = 256 / M, kblocks = (p->Kh + cpw - 1) / cpw;
        for (int gi = 0; gi < p->ngroups; ++gi) {
            p->boff[gi] = total;
            p->bcount[gi] = (size_t)p->Kh * M * L * p->gsize[gi];
            total += p->bcount[gi];
            p->boff32[gi] = total32;
            total32 += (size_t)kblocks * L * p->gsize[gi] * 256;
        }
#define PC_TRY(expr)                                                                                \
    {                                                                                               \
        hipError_t _e = (expr);                                                                     \
        if (_e != hipSuccess) {                                                                     \
            st = fail(SAFR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));            \
            break;                                                                                  \
        }                                                                                           \
    }
        PC_TRY(hipMalloc(&p->B64, total * sizeof(double2)));
        PC_TRY(hipMalloc(&p->B32, total32 * sizeof(float2)));
        PC_TRY(hipMemsetAsync(p->B32, 0, total32 * sizeof(float2), stream));
        if (p->mixed) {
            std::vector<double2> X, Y;
            tt_transforms(pup, n, M, p->p0, X, Y);
            std::vector<float2> Xf(X.size()), Yf(Y.size());
            for (size_t i = 0; i < X.size(); ++i) {
                Xf[i] = make_float2((float)X[i].x, (float)X[i].y);
                Yf[i] = make_float2((float)Y[i].x, (float)Y[i].y);
            }
            PC_TRY(hipMalloc(&p->Xh, Xf.size() * sizeof(float2)));
            PC_TRY(hipMalloc(&p->Yh, Yf.size() * sizeof(float2)));
            PC_TRY(hipMemcpy(p->Xh, Xf.data(), Xf.size() * sizeof(float2), hipMemcpyHostToDevice));
            PC_TRY(hipMemcpy(p->Yh, Yf.data(), Yf.size() * sizeof(float2), hipMemcpyHostToDevice));
            PC_TRY(hipMalloc(&p->X64, X.size() * sizeof(double2)));
            PC_TRY(hipMalloc(&p->Y64, Y.size() * sizeof(double2)));
            PC_TRY(hipMemcpy(p->X64, X.data(), X.size() * sizeof(double2), hipMemcpyHostToDevice));
            PC_TRY(hipMemcpy(p->Y64, Y.data(), Y.size() * sizeof(double2), hipMemcpyHostToDevice));
        }
        std::vector<float2> tw(M);
        for (int e = 0; e < M; ++e)
            tw[e] = make_float2((float)std::cos(2.0 * M_PI * e / M), (float)std::sin(2.0 * M_PI * e / M));
        PC_TRY(hipMalloc(&p->tw, M * sizeof(float2)));
        PC_TRY(hipMemcpy(p->tw, tw.data(), M * sizeof(float2), hipMemcpyHostToDevice));
        PC_TRY(hipMalloc(&p->pupil, pup.size()));
        PC_TRY(hipMemcpy(p->pupil, pup.data(), pup.size(), hipMemcpyHostToDevice));
        for (int g = 0; g < J; ++g) p->tt_mode[g] = mode[g];
        {
            // closed loop: star g's line of sight through pupil pixel (i, j) crosses output layer l at
            // c^s_l r + theta_g h_l, r = (p0 + i - M/2, p0 + j - M/2) pitch; on the layer grid (spacing
            // c_l pitch, centred at M/2) that is (u0 + m i, v0 + m j) with m = c^s_l / c_l
            std::vector<float4> tab((size_t)J * L);
            for (int g = 0; g < J; ++g)
                for (int l = 0; l < L; ++l) {
                    const safr_star& st = geo->stars[g];
                    const double cs = st.kind == SAFR_LGS ? 1.0 - heights[l] / geo->h_lgs : 1.0;
                    const double co = p->c_out[l];
                    const double m = cs / co, base = m * (p->p0 - 0.5 * M) + 0.5 * M;
                    const double sx = st.ax * heights[l] / (co * geo->pitch);
                    const double sy = st.ay * heights[l] / (co * geo->pitch);
                    tab[(size_t)g * L + l] = make_float4((float)m, (float)(base + sx), (float)(base + sy), 0.f);
                }
            PC_TRY(hipMalloc(&p->polc_tab, tab.size() * sizeof(float4)));
            PC_TRY(hipMemcpy(p->polc_tab, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice));
        }
        PC_TRY(hipMalloc(&dbad, sizeof(int)));
        PC_TRY(hipMemsetAsync(dbad, 0, sizeof(int), stream));
        const int H = p->Kh * M;
        int gmax = std::max(p->gsize[0], p->gsize[1]);
        const int Cm = std::min(gmax, L);
        if (geo->filter == SAFR_FILTER_MLP) {
            PC_TRY(hipMalloc(&feats, (size_t)H * Cm * 4 * sizeof(float)));
            PC_TRY(hipMalloc(&phi, (size_t)H * Cm * sizeof(float)));
            PC_TRY(hipMalloc(&mlp_dev, SAFR_MLP_PARAMS * sizeof(float)));
            PC_TRY(hipMemcpy(mlp_dev, geo->mlp, SAFR_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
        }
        if (geo->alpha_weight) {
            PC_TRY(hipMalloc(&aw_dev, (size_t)M * M * sizeof(double)));
            PC_TRY(hipMemcpy(aw_dev, geo->alpha_weight, (size_t)M * M * sizeof(double), hipMemcpyHostToDevice));
        }
        for (int gi = 0; gi < p->ngroups && st == SAFR_OK; ++gi) {
            PrecompArgs a{};
            a.M = M;
            a.G = p->gsize[gi];
            a.L = L;
            a.T = p->T;
            a.beta = geo->beta;
            a.alpha = p->galpha[gi];
            for (int m = 0; m < a.G; ++m) {
                a.ax[m] = geo->stars[p->gstar[gi][m]].ax;
                a.ay[m] = geo->stars[p->gstar[gi][m]].ay;
            }
            for (int l = 0; l < L; ++l) {
                a.h[l] = heights[l];
                a.c[l] = cgrp[gi][l];
                a.gamma[l] = weights[l] / wsum;
                a.sqrt_gamma[l] = std::sqrt(weights[l] / wsum);
            }
            {
                const int R = std::max(a.G, L), C = std::min(a.G, L);
                PC_TRY(hipMalloc(&a.W, (size_t)H * R * C * sizeof(double2)));
                PC_TRY(hipMalloc(&a.Q, (size_t)H * C * C * sizeof(double2)));
                PC_TRY(hipMalloc(&a.sigma, (size_t)H * C * sizeof(double)));
                p->pre[gi].W = a.W;                      // owned by the plan from here on
                p->pre[gi].Q = a.Q;
                p->pre[gi].sigma = a.sigma;
            }
            a.feats = feats;
            a.phi = phi;
            a.B64 = p->B64 + p->boff[gi];
            a.B32 = p->B32 + p->boff32[gi];
            a.log10_noise = geo->filter == SAFR_FILTER_MLP ? std::log10(geo->noise) : 0.0;
            a.bad = dbad;
            a.tsvd = geo->filter == SAFR_FILTER_TSVD;
            a.aw = aw_dev;
            PC_TRY(launch_svd(a, stream));
            if (geo->filter == SAFR_FILTER_MLP) {
                const int C = std::min(a.G, L);
                PC_TRY(launch_mlp_infer(mlp_dev, feats, phi, H * C, (float)a.log10_noise, stream));
            }
            PC_TRY(launch_assemble(a, stream));
            p->pre[gi] = a;                              // geometry and SVD; temporaries cleared below
            p->pre[gi].feats = nullptr;
            p->pre[gi].phi = nullptr;
            p->pre[gi].bad = nullptr;
            p->pre[gi].aw = nullptr;
        }
        if (st != SAFR_OK) break;
        p->filter = geo->filter;
        p->weighted = geo->alpha_weight != nullptr;
        int hbad = 0;
        PC_TRY(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, stream));
        PC_TRY(hipStreamSynchronize(stream));
        if (hbad) {
            st = fail(SAFR_ERR_NUMERIC, "non-finite value in the precomputed operator");
            break;
        }
        if (p->mixed) {
            st = build_basis(p, stream);
            if (st != SAFR_OK) break;
        }
        st = build_pack(p, stream);
        if (st != SAFR_OK) break;
        p->ws_own_bytes = ws_bytes(p, 1);
        PC_TRY(hipMalloc(&p->ws_own, p->ws_own_bytes));
        PC_TRY(hipMalloc(&p->dfirst, sizeof(int)));
        {
            const char* env = std::getenv("SAFR_CHECK_FINITE");
            p->check_finite = env && env[0] == '1';
        }
        PC_TRY(hipStreamSynchronize(stream));
#undef PC_TRY
    } while (0);
    (void)hipFree(feats);
    (void)hipFree(phi);
    (void)hipFree(mlp_dev);
    (void)hipFree(aw_dev);
    (void)hipFree(dbad);
    if (st != SAFR_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    return SAFR_OK;
}

safr_status safr_workspace_size(const safr_plan* p, int frames, int precision, size_t* bytes) {
    if (!p || !bytes) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    *bytes = ws_bytes(p, frames);
    return SAFR_OK;
}

safr_status safr_set_workspace(safr_plan* p, void* dev, size_t bytes) {
    if (!p) return fail(SAFR_ERR_ARG, "plan is NULL");
    if (dev && (reinterpret_cast<uintptr_t>(dev) & 255)) return fail(SAFR_ERR_ARG, "workspace not 256-byte aligned");
    if (dev != p->ws_user || (dev ? bytes : 0) != p->ws_user_bytes) drop_graphs(p);   // graphs hold workspace addresses
    p->ws_user = dev;
    p->ws_user_bytes = dev ? bytes : 0;
    return SAFR_OK;
}

safr_status safr_plan_info(const safr_plan* p, safr_plan_desc* d) {
    if (!p || !d) return fail(SAFR_ERR_ARG, "NULL argument");
    std::memset(d, 0, sizeof(*d));
    d->n = p->n;
    d->M = p->M;
    d->J = p->J;
    d->L = p->L;
    d->groups = p->ngroups;
    for (int gi = 0; gi < p->ngroups; ++gi) {
        d->group_size[gi] = p->gsize[gi];
        d->group_kind[gi] = p->gkind[gi];
        d->B_complex_per_group[gi] = p->bcount[gi];
    }
    for (int l = 0; l < p->L; ++l) {
        d->c[l] = p->c_out[l];
        d->layer_pitch[l] = p->c_out[l] * p->pitch;
    }
    return SAFR_OK;
}

safr_status safr_export_B(const safr_plan* p, int group, double* host, size_t count) {
    if (!p || !host) return fail(SAFR_ERR_ARG, "NULL argument");
    if (group < 0 || group >= p->ngroups) return fail(SAFR_ERR_ARG, "bad group %d", group);
    const size_t need = 2 * p->bcount[group];
    if (count < need) return fail(SAFR_ERR_ARG, "buffer holds %zu doubles, need %zu", count, need);
    // device layout [k][l][g][j] -> export layout [k][j][l][g]
    std::vector<double2> tmp(p->bcount[group]);
    HIP_TRY(hipMemcpy(tmp.data(), p->B64 + p->boff[group], tmp.size() * sizeof(double2),
                      hipMemcpyDeviceToHost));
    const int M = p->M, L = p->L, G = p->gsize[group];
    for (int k = 0; k < p->Kh; ++k)
        for (int l = 0; l < L; ++l)
            for (int g = 0; g < G; ++g)
                for (int j = 0; j < M; ++j) {
                    const double2 v = tmp[(((size_t)k * L + l) * G + g) * M + j];
                    const size_t o = (((size_t)k * M + j) * L + l) * G + g;
                    host[2 * o] = v.x;
                    host[2 * o + 1] = v.y;
                }
    return SAFR_OK;
}

safr_status safr_import_B(safr_plan* p, int group, const double* host, size_t count, hipStream_t s) {
    if (!p || !host) return fail(SAFR_ERR_ARG, "NULL argument");
    if (group < 0 || group >= p->ngroups) return fail(SAFR_ERR_ARG, "bad group %d", group);
    const size_t need = 2 * p->bcount[group];
    if (count != need) return fail(SAFR_ERR_ARG, "B of group %d holds %zu doubles, got %zu", group, need, count);
    for (size_t i = 0; i < need; ++i)
        if (!std::isfinite(host[i])) return fail(SAFR_ERR_NUMERIC, "non-finite value at %zu", i);
    // export layout [k][j][l][g] -> device FP64 [k][l][g][j] and the FP32 column-pass layout
    // [k / CPW][l][g][k % CPW][j] with the 1/M^2 of IDFT2 folded in (the precompute's own arithmetic)
    const int M = p->M, L = p->L, G = p->gsize[group], Kh = p->Kh, cpw = 256 / M;
    const int kblocks = (Kh + cpw - 1) / cpw;
    std::vector<double2> b64(p->bcount[group]);
    std::vector<float2> b32((size_t)kblocks * L * G * 256, make_float2(0.f, 0.f));
    const double inv_m2 = 1.0 / ((double)M * (double)M);
    for (int k = 0; k < Kh; ++k)
        for (int j = 0; j < M; ++j)
            for (int l = 0; l < L; ++l)
                for (int g = 0; g < G; ++g) {
                    const size_t i = (((size_t)k * M + j) * L + l) * G + g;
                    const double2 v = make_double2(host[2 * i], host[2 * i + 1]);
                    b64[(((size_t)k * L + l) * G + g) * M + j] = v;
                    b32[((((size_t)(k / cpw) * L + l) * G + g) * cpw + (k % cpw)) * M + j] =
                        make_float2((float)(v.x * inv_m2), (float)(v.y * inv_m2));
                }
    HIP_TRY(hipStreamSynchronize(s));          // work issued before the import uses the old operator
    HIP_TRY(hipMemcpy(p->B64 + p->boff[group], b64.data(), b64.size() * sizeof(double2), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->B32 + p->boff32[group], b32.data(), b32.size() * sizeof(float2), hipMemcpyHostToDevice));
    if (group == 1) {
        const safr_status st = build_basis(p, s);
        if (st != SAFR_OK) return st;
    } else {
        const safr_status st = build_pack(p, s);
        if (st != SAFR_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(s));
    p->imported = 1;
    return SAFR_OK;
}

safr_status safr_deadline_stats(safr_plan* p, safr_deadline_info* out, int reset, hipStream_t s) {
    if (!p || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->period_us = p->deadline_us;
    if (!p->dstats) return SAFR_OK;
    unsigned long long h[5] = {0, 0, 0, 0, 0};
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(h, p->dstats, sizeof(h), hipMemcpyDeviceToHost));
    out->steps = h[0];
    out->misses = h[1];
    out->last_us = h[2] / p->ticks_per_us;
    out->max_us = h[3] / p->ticks_per_us;
    if (reset) HIP_TRY(hipMemset(p->dstats, 0, sizeof(h)));
    return SAFR_OK;
}

safr_status safr_update_alpha(safr_plan* p, double alpha, double alpha_tt, int filter, const double* alpha_weight,
                              hipStream_t s) {
    if (!p) return fail(SAFR_ERR_ARG, "plan is NULL");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SAFR_ERR_ARG, "alpha must be >= 0");
    if (!(alpha_tt >= 0.0) || !std::isfinite(alpha_tt)) return fail(SAFR_ERR_ARG, "alpha_tt must be >= 0");
    if (filter != SAFR_FILTER_TIKHONOV && filter != SAFR_FILTER_TSVD)
        return fail(SAFR_ERR_ARG, "a refresh takes the Tikhonov or TSVD filter");
    if (alpha_weight) {
        const safr_status ws = check_alpha_weight(p->M, alpha_weight);
        if (ws != SAFR_OK) return ws;
    }
    const int M = p->M;
    const double galpha[2] = {alpha, p->mixed ? alpha_tt : 0.0};
    // the natural group (and its basis images) changes only with alpha_tt, the filter or a weight map
    const bool redo1 = p->mixed && (alpha_tt != p->galpha[1] || filter != p->filter || alpha_weight || p->weighted);
    safr_status st = SAFR_OK;
    double* aw_dev = nullptr;
    int* dbad = nullptr;
    do {
        const int clear = 0;
        BT_TRY(hipMalloc(&dbad, sizeof(int)));
        BT_TRY(hipMemcpyAsync(dbad, &clear, sizeof(int), hipMemcpyHostToDevice, s));
        if (alpha_weight) {
            BT_TRY(hipMalloc(&aw_dev, (size_t)M * M * sizeof(double)));
            BT_TRY(hipMemcpy(aw_dev, alpha_weight, (size_t)M * M * sizeof(double), hipMemcpyHostToDevice));
        }
        for (int gi = 0; gi < p->ngroups; ++gi) {
            if (gi == 1 && !redo1) continue;
            PrecompArgs a = p->pre[gi];
            a.alpha = galpha[gi];
            a.tsvd = filter == SAFR_FILTER_TSVD;
            a.aw = aw_dev;
            a.phi = nullptr;
            a.bad = dbad;
            BT_TRY(launch_assemble(a, s));
        }
        if (st != SAFR_OK) break;
        int hbad = 0;
        BT_TRY(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, s));
        BT_TRY(hipStreamSynchronize(s));
        if (hbad) {
            st = fail(SAFR_ERR_NUMERIC, "non-finite value in the refreshed operator");
            break;
        }
        if (redo1) {
            st = build_basis(p, s);
            if (st != SAFR_OK) break;
        }
        st = build_pack(p, s);
        if (st != SAFR_OK) break;
        BT_TRY(hipStreamSynchronize(s));
        p->galpha[0] = galpha[0];
        p->galpha[1] = galpha[1];
        p->filter = filter;
        p->weighted = alpha_weight != nullptr;
        p->imported = 0;
    } while (0);
    (void)hipFree(aw_dev);
    (void)hipFree(dbad);
    return st;
}

safr_status safr_reconstruct_batched(safr_plan* p, int frames, const float* wf, float* out, int precision,
                                     hipStream_t s) {
    if (!p || !wf || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    if (precision == SAFR_BF16X3 && !p->Apack)
        return fail(SAFR_ERR_UNSUPPORTED, "BF16 path not available for this plan");
    const size_t need = ws_bytes(p, frames);
    void* ws = nullptr;
    if (p->ws_user && p->ws_user_bytes >= need) ws = p->ws_user;
    else if (p->ws_own_bytes >= need) ws = p->ws_own;
    else return fail(SAFR_ERR_STATE, "workspace of %zu bytes needed for %d frames", need, frames);
    if (p->check_finite) {
        const safr_status cs = check_inputs(p, frames, wf, nullptr, s);
        if (cs != SAFR_OK) return cs;
        return launch_all(p, frames, wf, out, precision, ws, s);
    }

    if (p->use_graph && s != nullptr) {
        const bool hit = p->gexec && p->g_frames == frames && p->g_prec == precision && p->g_wf == wf &&
                         p->g_out == out && p->g_stream == s;
        if (!hit) {
            if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
            if (p->graph) (void)hipGraphDestroy(p->graph);
            p->gexec = nullptr;
            p->graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            safr_status st = launch_all(p, frames, wf, out, precision, ws, s);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (st != SAFR_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(SAFR_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            p->graph = g;
            HIP_TRY(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
            p->g_frames = frames;
            p->g_prec = precision;
            p->g_wf = wf;
            p->g_out = out;
            p->g_stream = s;
        }
        HIP_TRY(hipGraphLaunch(p->gexec, s));
        return SAFR_OK;
    }
    return launch_all(p, frames, wf, out, precision, ws, s);
}

safr_status safr_reconstruct(safr_plan* p, const float* wf, float* out, hipStream_t s) {
    return safr_reconstruct_batched(p, 1, wf, out, SAFR_FP32, s);
}

}  // extern "C"

namespace {

// Workspace of safr_reconstruct_batched_static: a file-scope device array (each GPU that loads the library
// holds its own copy until the process ends).  In host code its name is only a stand-in: the device address
// is looked up once per device with hipGetSymbolAddress and kept; kernels receive that address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

safr_status static_scratch(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAFR_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SAFR_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SAFR_OK;
}

}  // namespace

extern "C" {

size_t safr_static_workspace_bytes(void) { return kStaticScratchBytes; }

safr_status safr_reconstruct_batched_static(safr_plan* p, int frames, const float* wf, float* out, int precision,
                                            hipStream_t s) {
    if (!p || !wf || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    if (precision == SAFR_BF16X3 && !p->Apack)
        return fail(SAFR_ERR_UNSUPPORTED, "BF16 path not available for this plan");
    const size_t need = ws_bytes(p, frames);
    if (need > kStaticScratchBytes)
        return fail(SAFR_ERR_ARG, "%d frames of this plan need %zu bytes of workspace; the static workspace holds %zu "
                                  "(at most %zu frames)", frames, need, kStaticScratchBytes,
                    (size_t)(kStaticScratchBytes / std::max<size_t>(1, ws_bytes(p, 1))));
    void* ws = nullptr;
    const safr_status st = static_scratch(&ws);
    if (st != SAFR_OK) return st;
    return launch_all(p, frames, wf, out, precision, ws, s);
}



safr_status safr_polc(safr_plan* p, int frames, const float* wf, const float* layers, float weight, float* out,
                      hipStream_t s) {
    if (!p || !wf || !layers || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (!std::isfinite(weight)) return fail(SAFR_ERR_ARG, "weight must be finite");
    HIP_TRY(launch_polc(polc_args(p, wf, layers, weight, out), frames, s));
    return SAFR_OK;
}

safr_status safr_strehl(safr_plan* p, int frames, int D, const double* dirs, const float* open_loop,
                        const float* layers, float scale, float* sr, float* var, hipStream_t s) {
    if (!p || !dirs || !open_loop || !layers || !sr) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (D < 1 || D > kMaxDirs) return fail(SAFR_ERR_ARG, "directions must be in 1..%d", kMaxDirs);
    if (!std::isfinite(scale)) return fail(SAFR_ERR_ARG, "scale must be finite");
    StrehlArgs a{};
    for (int d = 0; d < D; ++d) {
        if (!std::isfinite(dirs[2 * d]) || !std::isfinite(dirs[2 * d + 1]))
            return fail(SAFR_ERR_ARG, "direction %d is not finite", d);
        a.dx[d] = (float)dirs[2 * d];
        a.dy[d] = (float)dirs[2 * d + 1];
    }
    for (int l = 0; l < p->L; ++l) {
        const double m = 1.0 / p->c_out[l];
        a.m[l] = (float)m;
        a.base[l] = (float)(m * (p->p0 - 0.5 * p->M) + 0.5 * p->M);
        a.hs[l] = (float)(p->heights[l] / (p->c_out[l] * p->pitch));
    }
    a.open_loop = open_loop;
    a.layers = layers;
    a.sr = sr;
    a.var = var;
    a.pupil = p->pupil;
    a.scale2 = scale * scale;
    a.n = p->n;
    a.M = p->M;
    a.L = p->L;
    a.D = D;
    const size_t need = (size_t)frames * D * strehl_chunks(p->n) * 3;
    if (p->strehl_part_floats < need) {          // grown on demand (synchronises the device once)
        HIP_TRY(hipStreamSynchronize(s));
        (void)hipFree(p->strehl_part);
        p->strehl_part = nullptr;
        p->strehl_part_floats = 0;
        HIP_TRY(hipMalloc(&p->strehl_part, need * sizeof(float)));
        p->strehl_part_floats = need;
    }
    a.part = p->strehl_part;
    HIP_TRY(launch_strehl(a, frames, s));
    return SAFR_OK;
}

safr_status safr_loop_step(safr_plan* p, int frames, const float* wf, const float* a_in, float gain, float* a_out,
                           hipStream_t s) {
    if (!p || !wf || !a_in || !a_out) return fail(SAFR_ERR_ARG, "NULL argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (!std::isfinite(gain)) return fail(SAFR_ERR_ARG, "gain must be finite");
    const size_t need = ws_bytes(p, frames);
    void* ws = nullptr;
    if (p->ws_user && p->ws_user_bytes >= need) ws = p->ws_user;
    else if (p->ws_own_bytes >= need) ws = p->ws_own;
    else return fail(SAFR_ERR_STATE, "workspace of %zu bytes needed for %d frames", need, frames);
    if (p->check_finite) {
        const safr_status cs = check_inputs(p, frames, wf, a_in, s);
        if (cs != SAFR_OK) return cs;
        return launch_loop(p, frames, wf, a_in, gain, a_out, ws, s);
    }

    if (p->use_graph && s != nullptr) {
        const bool hit = p->lexec && p->l_frames == frames && p->l_gain == gain && p->l_wf == wf &&
                         p->l_ain == a_in && p->l_aout == a_out && p->l_stream == s;
        if (!hit) {
            if (p->lexec) (void)hipGraphExecDestroy(p->lexec);
            if (p->lgraph) (void)hipGraphDestroy(p->lgraph);
            p->lexec = nullptr;
            p->lgraph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            safr_status st = launch_loop(p, frames, wf, a_in, gain, a_out, ws, s);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (st != SAFR_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(SAFR_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            p->lgraph = g;
            HIP_TRY(hipGraphInstantiate(&p->lexec, g, nullptr, nullptr, 0));
            p->l_frames = frames;
            p->l_gain = gain;
            p->l_wf = wf;
            p->l_ain = a_in;
            p->l_aout = a_out;
            p->l_stream = s;
        }
        HIP_TRY(hipGraphLaunch(p->lexec, s));
        return SAFR_OK;
    }
    return launch_loop(p, frames, wf, a_in, gain, a_out, ws, s);
}

safr_status safr_time_stages(safr_plan* p, int frames, const float* wf, float* out, int precision, int iters,
                             hipStream_t s, double* ms) {
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (!p || !wf || !out || !ms || iters < 1) return fail(SAFR_ERR_ARG, "bad argument");
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    if (precision == SAFR_BF16X3 && !p->Apack) return fail(SAFR_ERR_UNSUPPORTED, "BF16 path not available");
    const size_t need = ws_bytes(p, frames);
    void* ws = nullptr;
    if (p->ws_user && p->ws_user_bytes >= need) ws = p->ws_user;
    else if (p->ws_own_bytes >= need) ws = p->ws_own;
    else return fail(SAFR_ERR_STATE, "workspace of %zu bytes needed for %d frames", need, frames);
    // one full sequence leaves every stage's inputs in the workspace; then each stage's launches run `iters`
    // times back to back between two events (no host synchronisation until the end)
    hipEvent_t ev[6] = {};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    safr_status st = launch_all(p, frames, wf, out, precision, ws, s);
    for (int k = 0; k < 3 && st == SAFR_OK; ++k) {
        if (hipEventRecord(ev[2 * k], s) != hipSuccess) st = fail(SAFR_ERR_DEVICE, "event record failed");
        for (int it = 0; it < iters && st == SAFR_OK; ++it)
            st = launch_all(p, frames, wf, out, precision, ws, s, nullptr, nullptr, 1.f, k);
        if (st == SAFR_OK && hipEventRecord(ev[2 * k + 1], s) != hipSuccess) st = fail(SAFR_ERR_DEVICE, "event record failed");
    }
    if (st == SAFR_OK && hipEventSynchronize(ev[5]) != hipSuccess) st = fail(SAFR_ERR_DEVICE, "event synchronisation failed");
    for (int k = 0; k < 3 && st == SAFR_OK; ++k) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) st = fail(SAFR_ERR_DEVICE, "event timing failed");
        ms[k] = (double)t / iters;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st;
}

namespace {

// average milliseconds of one stage over `iters` synchronised launches of the whole sequence
safr_status time_stage(safr_plan* p, int frames, const float* wf, float* out, int precision, void* ws, int iters,
                       hipStream_t s, hipEvent_t* ev, int stage, double* ms) {
    double acc = 0.0;
    for (int it = 0; it < iters; ++it) {
        safr_status st = launch_all(p, frames, wf, out, precision, ws, s, ev);
        if (st != SAFR_OK) return st;
        if (hipEventSynchronize(ev[3]) != hipSuccess) return fail(SAFR_ERR_DEVICE, "event synchronisation failed");
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ev[stage], ev[stage + 1]));
        acc += t;
    }
    *ms = acc / iters;
    return SAFR_OK;
}

}  // namespace

safr_status safr_autotune(safr_plan* p, int frames, const float* wf, float* out, int precision, int iters,
                          hipStream_t s, int* choice) {
    if (!p || !wf || !out || iters < 1) return fail(SAFR_ERR_ARG, "bad argument");
    if (frames < 1 || frames > kMaxFrames) return fail(SAFR_ERR_ARG, "frames must be in 1..%d", kMaxFrames);
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    if (precision == SAFR_BF16X3 && !p->Apack) return fail(SAFR_ERR_UNSUPPORTED, "BF16 path not available");
    const size_t need = ws_bytes(p, frames);
    void* ws = nullptr;
    if (p->ws_user && p->ws_user_bytes >= need) ws = p->ws_user;
    else if (p->ws_own_bytes >= need) ws = p->ws_own;
    else return fail(SAFR_ERR_STATE, "workspace of %zu bytes needed for %d frames", need, frames);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    safr_status st = SAFR_OK;
    const int T = team_size(p->M);
    // row pass: transform teams per block (powers of two, and the counts that split the pupil rows into
    // equal chunks)
    {
        int best = p->row_teams;
        double bt = 1e30;
        std::vector<int> cand = {1, 2, 4, 8, 16};
        const int npairs = (p->n + 1) / 2;
        for (int c = 1; c <= npairs; ++c) cand.push_back((npairs + c - 1) / c);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int teams : cand) {
            if (teams * T > 256 || rows_lds_bytes(p->M, p->n, teams) > kMaxLds || 2 * teams > 2 * p->n) continue;
            p->row_teams = teams;
            double ms = 0.0;
            if ((st = time_stage(p, frames, wf, out, precision, ws, iters, s, ev, 0, &ms)) != SAFR_OK) break;
            if (ms < bt) { bt = ms; best = teams; }
        }
        p->row_teams = best;
    }
    // output pass: rows per block, then frames per block (multiples of the frames one iteration transforms)
    if (st == SAFR_OK) {
        int best = p->out_rows, bestf = p->out_frames;
        double bt = 1e30;
        for (int rows : {8, 16, 32}) {
            if (!out_rows_supported(p->M, rows) || out_lds_bytes(p->M, rows, p->nb) > kMaxLds) continue;
            const int nf = out_frames_per_iter(p->M, rows);
            for (int mult : {1, 2, 4, 8, 16}) {
                if (mult > 1 && nf * mult / 2 >= frames) break;
                p->out_rows = rows;
                p->out_frames = nf * mult;
                double ms = 0.0;
                if ((st = time_stage(p, frames, wf, out, precision, ws, iters, s, ev, 2, &ms)) != SAFR_OK) break;
                if (ms < bt) {
                    bt = ms;
                    best = rows;
                    bestf = nf * mult;
                }
            }
            if (st != SAFR_OK) break;
        }
        p->out_rows = best;
        p->out_frames = bestf;
    }
    // column pass (FP32): frames transformed together (B read once for them) and frames per block
    if (st == SAFR_OK && precision == SAFR_FP32) {
        int best = p->col_frames, bestn = p->col_nf;
        double bt = 1e30;
        const bool fixed = p->col_prefetch && cols_fixed_shape(p->M, p->L, p->gsize[0], p->mixed ? 1 : 0);
        p->col_frames_auto = 0;                           // the candidates below are timed as set
        for (int nf : {1, 2, 4}) {
            if (nf > 1 && (!fixed || nf > frames)) break;
            if (cols_lds_bytes(p->M, p->gsize[0], p->L, nf, fixed) > kMaxLds) break;
            for (int mult : {1, 2, 4, 8}) {
                const int cf = nf * mult;
                if (mult > 1 && cf / 2 >= frames) break;
                p->col_nf = nf;
                p->col_frames = cf;
                double ms = 0.0;
                if ((st = time_stage(p, frames, wf, out, precision, ws, iters, s, ev, 1, &ms)) != SAFR_OK) break;
                if (ms < bt) {
                    bt = ms;
                    best = cf;
                    bestn = nf;
                }
            }
            if (st != SAFR_OK) break;
        }
        p->col_frames = best;
        p->col_nf = bestn;
        p->col_frames_auto = 0;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    drop_graphs(p);
    if (choice) {
        choice[0] = p->row_teams;
        choice[1] = p->out_rows;
        choice[2] = p->col_frames;
        choice[3] = p->out_frames;
        choice[4] = p->col_nf;
    }
    return st;
}

void safr_destroy(safr_plan* p) { free_plan(p); }

}  // extern "C"

struct safr_multi {
    int count = 0, precision = SAFR_FP32;
    std::vector<safr_plan*> plans;
    std::vector<int> frames;
    std::vector<void*> ws;
    std::vector<hipStream_t> side;          // one per entry after the first
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const float*> g_wf;
    std::vector<float*> g_out;
    hipStream_t g_stream = nullptr;
};

namespace {

void free_multi(safr_multi* m) {
    if (!m) return;
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    for (void* w : m->ws) (void)hipFree(w);
    for (hipStream_t st : m->side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : m->done) (void)hipEventDestroy(e);
    if (m->fork) (void)hipEventDestroy(m->fork);
    delete m;
}

// every entry's launch sequence, entry 0 on `s`, the others on side streams forked from and joined to `s`
safr_status multi_launch(safr_multi* m, const float* const* wf, float* const* out, hipStream_t s) {
    HIP_TRY(hipEventRecord(m->fork, s));
    for (int i = 1; i < m->count; ++i) {
        HIP_TRY(hipStreamWaitEvent(m->side[i - 1], m->fork, 0));
        safr_status st = launch_all(m->plans[i], m->frames[i], wf[i], out[i], m->precision, m->ws[i], m->side[i - 1]);
        if (st != SAFR_OK) return st;
        HIP_TRY(hipEventRecord(m->done[i - 1], m->side[i - 1]));
    }
    safr_status st = launch_all(m->plans[0], m->frames[0], wf[0], out[0], m->precision, m->ws[0], s);
    if (st != SAFR_OK) return st;
    for (int i = 1; i < m->count; ++i) HIP_TRY(hipStreamWaitEvent(s, m->done[i - 1], 0));
    return SAFR_OK;
}

}  // namespace

extern "C" {

safr_status safr_multi_create(safr_plan* const* plans, const int* frames, int count, int precision,
                              safr_multi** out) {
    if (!out) return fail(SAFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || !frames || count < 1) return fail(SAFR_ERR_ARG, "need at least one plan");
    if (precision != SAFR_FP32 && precision != SAFR_BF16X3) return fail(SAFR_ERR_ARG, "bad precision");
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || frames[i] < 1 || frames[i] > kMaxFrames)
            return fail(SAFR_ERR_ARG, "entry %d: bad plan or frame count", i);
        if (precision == SAFR_BF16X3 && !plans[i]->Apack)
            return fail(SAFR_ERR_UNSUPPORTED, "entry %d: BF16 path not available for its plan", i);
    }
    safr_multi* m = new safr_multi();
    m->count = count;
    m->precision = precision;
    for (int i = 0; i < count; ++i) {
        m->plans.push_back(plans[i]);
        m->frames.push_back(frames[i]);
        void* w = nullptr;
        hipError_t e = hipMalloc(&w, ws_bytes(plans[i], frames[i]));
        if (e != hipSuccess) {
            free_multi(m);
            return fail(SAFR_ERR_DEVICE, "workspace allocation failed: %s", hipGetErrorString(e));
        }
        m->ws.push_back(w);
        if (i > 0) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                free_multi(m);
                return fail(SAFR_ERR_DEVICE, "stream or event creation failed");
            }
            m->side.push_back(st);
            m->done.push_back(ev);
        }
    }
    if (hipEventCreateWithFlags(&m->fork, hipEventDisableTiming) != hipSuccess) {
        free_multi(m);
        return fail(SAFR_ERR_DEVICE, "event creation failed");
    }
    *out = m;
    return SAFR_OK;
}

safr_status safr_multi_execute(safr_multi* m, const float* const* wf, float* const* out, hipStream_t s) {
    if (!m || !wf || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    for (int i = 0; i < m->count; ++i)
        if (!wf[i] || !out[i]) return fail(SAFR_ERR_ARG, "entry %d: NULL buffer", i);
    if (s == nullptr) return multi_launch(m, wf, out, s);       // the legacy stream cannot be captured
    bool hit = m->exec && m->g_stream == s;
    for (int i = 0; hit && i < m->count; ++i) hit = m->g_wf[i] == wf[i] && m->g_out[i] == out[i];
    if (!hit) {
        if (m->exec) (void)hipGraphExecDestroy(m->exec);
        if (m->graph) (void)hipGraphDestroy(m->graph);
        m->exec = nullptr;
        m->graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        safr_status st = multi_launch(m, wf, out, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != SAFR_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(SAFR_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        m->graph = g;
        HIP_TRY(hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0));
        m->g_wf.assign(wf, wf + m->count);
        m->g_out.assign(out, out + m->count);
        m->g_stream = s;
    }
    HIP_TRY(hipGraphLaunch(m->exec, s));
    return SAFR_OK;
}

safr_status safr_multi_autotune(safr_multi* m, const float* const* wf, float* const* out, int iters, hipStream_t s) {
    if (!m || !wf || !out) return fail(SAFR_ERR_ARG, "NULL argument");
    for (int i = 0; i < m->count; ++i) {
        safr_plan* p = m->plans[i];
        void* save = p->ws_user;
        const size_t save_b = p->ws_user_bytes;
        p->ws_user = m->ws[i];
        p->ws_user_bytes = ws_bytes(p, m->frames[i]);
        safr_status st = safr_autotune(p, m->frames[i], wf[i], out[i], m->precision, iters, s, nullptr);
        p->ws_user = save;
        p->ws_user_bytes = save_b;
        if (st != SAFR_OK) return st;
    }
    if (m->exec) {
        (void)hipGraphExecDestroy(m->exec);
        (void)hipGraphDestroy(m->graph);
        m->exec = nullptr;
        m->graph = nullptr;
    }
    return SAFR_OK;
}

void safr_multi_destroy(safr_multi* m) { free_multi(m); }

safr_status safr_set_option(safr_plan* p, int option, int value) {
    if (!p) return fail(SAFR_ERR_ARG, "plan is NULL");
    drop_graphs(p);
    switch (option) {
        case 0: p->use_graph = value != 0; return SAFR_OK;
        case 1:
            if (value < 1 || value * team_size(p->M) > 256) return fail(SAFR_ERR_ARG, "bad row team count");
            if (rows_lds_bytes(p->M, p->n, value) > kMaxLds)
                return fail(SAFR_ERR_ARG, "%d row teams need more than 160 KiB of LDS", value);
            p->row_teams = value;
            return SAFR_OK;
        case 2:
            if (!out_rows_supported(p->M, value))
                return fail(SAFR_ERR_ARG, "output rows per block must be 8, 16 or 32, at most M and at least 1024 / M");
            if (out_lds_bytes(p->M, value, p->nb) > kMaxLds)
                return fail(SAFR_ERR_ARG, "%d output rows per block need more than 160 KiB of LDS", value);
            p->out_rows = value;
            return SAFR_OK;
        case 3:
            if (value != 4 && value != 8 && value != 16) return fail(SAFR_ERR_ARG, "frames per MFMA block: 4, 8 or 16");
            if (!p->Apack) return fail(SAFR_ERR_UNSUPPORTED, "BF16 path not available for this plan");
            if (mfma_lds_bytes(p->M, value, p->gsize[0], p->L) > kMaxLds)
                return fail(SAFR_ERR_ARG, "%d frames per MFMA block need more than 160 KiB of LDS", value);
            p->mfma_frames = value;
            return SAFR_OK;
        case 4:
            if (value < 1 || value > 4096) return fail(SAFR_ERR_ARG, "bad frames per column block");
            p->col_frames = value;
            p->col_frames_auto = 0;
            return SAFR_OK;
        case 5: p->col_prefetch = value != 0; return SAFR_OK;
        case 6:
            if (value < 1 || value > 4096) return fail(SAFR_ERR_ARG, "bad frames per output block");
            p->out_frames = value;
            return SAFR_OK;
        case 7:
            if (value != 1 && value != 2 && value != 4)
                return fail(SAFR_ERR_ARG, "frames transformed together in the column pass: 1, 2 or 4");
            if (cols_lds_bytes(p->M, p->gsize[0], p->L, value, true) > kMaxLds)
                return fail(SAFR_ERR_ARG, "%d frames together need more than 160 KiB of LDS", value);
            p->col_nf = value;
            return SAFR_OK;
        case 8: p->check_finite = value != 0; return SAFR_OK;
        case 11:
            if (value < 0 || value > kMaxFrames) return fail(SAFR_ERR_ARG, "bad frames per launch sequence");
            p->seq_frames = value;
            return SAFR_OK;
        case 12: p->fused = value != 0; return SAFR_OK;
        case 10: {
            const int was = p->col_mfma;
            p->col_mfma = value != 0;
            if (p->col_mfma && !was) {      // the lane layout of B (kept up to date only while on)
                // work still in flight on any stream may read the copy being rewritten
                HIP_TRY(hipDeviceSynchronize());
                const safr_status st = build_mfma_b(p, nullptr);
                if (st != SAFR_OK) {
                    p->col_mfma = 0;
                    return st;
                }
                HIP_TRY(hipStreamSynchronize(nullptr));
            }
            return SAFR_OK;
        }
        case 9: {
            if (value < 0) return fail(SAFR_ERR_ARG, "the deadline must be >= 0 microseconds");
            if (value > 0 && !p->dstats) {
                int dev = 0, khz = 0;
                HIP_TRY(hipGetDevice(&dev));
                HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
                if (khz <= 0) return fail(SAFR_ERR_DEVICE, "no device wall clock");
                HIP_TRY(hipMalloc(&p->dstats, 5 * sizeof(unsigned long long)));
                HIP_TRY(hipMemset(p->dstats, 0, 5 * sizeof(unsigned long long)));
                p->ticks_per_us = khz / 1000.0;
            }
            p->deadline_us = value;
            p->deadline_ticks = value > 0 ? (unsigned long long)std::llround(value * p->ticks_per_us) : 0ull;
            return SAFR_OK;
        }
        default: return fail(SAFR_ERR_ARG, "unknown option %d", option);
    }
}

}  // extern "C"

namespace {

// one launch sequence (row, column and output pass) over `frames` frames
safr_status launch_seq(safr_plan* p, int frames, const float* wf, float* out, int precision, void* ws,
                       hipStream_t s, hipEvent_t* ev, const float* prev, float gain, int stage) {
    const bool do_rows = stage < 0 || stage == 0, do_cols = stage < 0 || stage == 1, do_out = stage < 0 || stage == 2;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    if (precision == SAFR_FP32 && p->fused && p->ngroups == 1 &&
        frame_shape(p->M, p->n, p->gsize[0], p->L, p->mixed ? 1 : 0)) {
        // the whole step in one kernel (counted as the row stage; the other two stages are empty)
        FrameArgs fa{};
        fa.wf = wf;
        fa.pupil = p->pupil;
        fa.tw = p->tw;
        fa.B = p->B32 + p->boff32[0];
        fa.out = out;
        fa.prev = prev;
        fa.gain = gain;
        fa.frames = frames;
        if (do_rows) HIP_TRY(launch_frame(fa, p->L, s));
        if (ev)
            for (int e = 1; e < 4; ++e) HIP_TRY(hipEventRecord(ev[e], s));
        return SAFR_OK;
    }
    char* base = reinterpret_cast<char*>(ws);
    float2* R = reinterpret_cast<float2*>(base);
    float2* C = reinterpret_cast<float2*>(base + ws_r(p, frames));
    float2* part = reinterpret_cast<float2*>(base + ws_r(p, frames) + ws_c(p, frames));
    float2* planes = reinterpret_cast<float2*>(base + ws_r(p, frames) + ws_c(p, frames) + ws_mom(p, frames));
    RowArgs ra{};
    ra.wf = wf;
    ra.R = R;
    ra.part = part;
    for (int i = 0; i < 3; ++i) {
        ra.tt_b[i] = p->tt_b[i];
        ra.tt_c[i] = p->tt_c[i];
    }
    ra.pupil = p->pupil;
    for (int g = 0; g < p->J; ++g) ra.tt_mode[g] = p->tt_mode[g];
    ra.tw = p->tw;
    ra.n = p->n;
    ra.J = p->J;
    ra.p0 = p->p0;
    ra.rows_per_block = 2 * p->row_teams;
    for (int gi = 0, slot = 0; gi < p->ngroups; ++gi)
        for (int m = 0; m < p->gsize[gi]; ++m) ra.slot[p->gstar[gi][m]] = slot++;
    const int nchunk = (p->n + ra.rows_per_block - 1) / ra.rows_per_block;
    if (do_rows) HIP_TRY(launch_rows(p->M, ra, frames, nchunk, p->row_teams, s));
    // split tomography: the passes add the row chunks' plane parts as they read them, or, for more chunks
    // than their lane groups take, read the sums of one more launch
    const float2* plane_src = part;
    int plane_nch = nchunk;
    if (p->mixed && nchunk > kPlaneLanes) {
        PlaneKArgs pk{};
        pk.part = part;
        pk.planes = planes;
        pk.nchunk = nchunk;
        pk.count = frames * p->J;
        if (do_rows) HIP_TRY(launch_planes(pk, s));
        plane_src = planes;
        plane_nch = 1;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));

    GroupArgs grp{};
    grp.G = p->gsize[0];
    grp.mode = p->mixed ? 1 : 0;
    if (precision == SAFR_FP32) {
        ColArgs ca{};
        ca.R = R;
        ca.B = p->B32 + p->boff32[0];
        ca.C = C;
        ca.tw = p->tw;
        ca.planes = plane_src;
        ca.plane_nch = plane_nch;
        ca.Xh = p->Xh;
        ca.Yh = p->Yh;
        ca.grp = grp;
        ca.n = p->n;
        ca.J = p->J;
        ca.L = p->L;
        ca.p0 = p->p0;
        ca.frames = frames;
        const bool fixed = p->col_prefetch && cols_fixed_shape(p->M, p->L, grp.G, grp.mode);
        int nf = fixed ? p->col_nf : 1;
        while (nf > 1 && nf > frames) nf /= 2;
        int fpb = p->col_frames;
        if (p->col_frames_auto) {
            // about two column blocks per CU, each looping over a multiple of the frames transformed together
            const int kblocks = (p->M / 2) / (256 / p->M);
            const int per = std::max(1, frames * kblocks / 512);
            fpb = std::max(nf, per / nf * nf);
        }
        ca.frames_per_block = std::max(1, std::min(fpb, frames));
        ca.prefetch = p->col_prefetch;
        ca.Bm = p->col_mfma ? p->Bm : nullptr;
        if (do_cols) HIP_TRY(launch_cols(p->M, ca, nf, frames, s));
    } else {
        MfmaArgs ma{};
        ma.R = R;
        ma.Apack = p->Apack;
        ma.C = C;
        ma.tw = p->tw;
        ma.grp = grp;
        ma.lt = p->mf_lt[0];
        ma.ntile = p->mf_ntile[0];
        ma.ppm = p->mf_ppm[0];
        ma.planes = plane_src;
        ma.plane_nch = plane_nch;
        ma.Xh = p->Xh;
        ma.Yh = p->Yh;
        ma.n = p->n;
        ma.J = p->J;
        ma.L = p->L;
        ma.p0 = p->p0;
        ma.frames = frames;
        if (do_cols) HIP_TRY(launch_cols_mfma(p->M, ma, frames, p->mfma_frames, s));
    }
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));

    OutArgs oa{};
    oa.C = C;
    oa.out = out;
    oa.tw = p->tw;
    oa.P = p->P;
    oa.planes = plane_src;
    oa.plane_nch = plane_nch;
    oa.nb = p->nb;
    oa.ngs_base = p->gsize[0];
    oa.L = p->L;
    oa.J = p->J;
    oa.frames = frames;
    oa.frames_per_block = std::max(1, p->out_frames);
    oa.prev = prev;
    oa.gain = gain;
    if (do_out) HIP_TRY(launch_out(p->M, oa, p->out_rows, frames, s));
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    return SAFR_OK;
}

// the call's frames in launch sequences of at most sequence_frames(p) frames, one after the other on the stream
// (each uses the start of the workspace; `ev`, when given, brackets the stages of the first sequence)
safr_status launch_all(safr_plan* p, int frames, const float* wf, float* out, int precision, void* ws,
                       hipStream_t s, hipEvent_t* ev, const float* prev, float gain, int stage) {
    const int cap = sequence_frames(p);
    if (frames <= cap) return launch_seq(p, frames, wf, out, precision, ws, s, ev, prev, gain, stage);
    const int nseq = (frames + cap - 1) / cap, per = (frames + nseq - 1) / nseq;
    const size_t wstride = (size_t)p->J * p->n * p->n, ostride = (size_t)p->L * p->M * p->M;
    for (int f0 = 0; f0 < frames; f0 += per) {
        const int nf = std::min(per, frames - f0);
        const safr_status st = launch_seq(p, nf, wf + f0 * wstride, out + f0 * ostride, precision, ws, s,
                                          f0 == 0 ? ev : nullptr, prev ? prev + f0 * ostride : nullptr, gain, stage);
        if (st != SAFR_OK) return st;
    }
    return SAFR_OK;
}

}  // namespace
