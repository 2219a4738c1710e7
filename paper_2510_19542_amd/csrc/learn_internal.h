// Internal definitions of the learned-filter kernels (training and inference).
#pragma once
#include "safr_internal.h"

namespace safr {

// planes of the per-row activation store act[plane][row]
enum : int {
    ACT_X = 0,          // 4 inputs
    ACT_A1 = 4,         // 64 GELU outputs of layer 1
    ACT_G1 = 68,        // 64 GELU derivatives of layer 1
    ACT_A2 = 132,
    ACT_G2 = 196,
    ACT_A3 = 260,
    ACT_G3 = 324,
    ACT_DZ1 = 388,      // 64 pre-activation gradients of layer 1
    ACT_DZ2 = 452,
    ACT_DZ3 = 516,
    ACT_DZ4 = 580,      // output pre-activation gradient
    ACT_PLANES = 581
};

// per-frequency constants (struct of arrays over the half spectrum h = k M + j)
struct LearnFreq {
    float2* U;          // [g][r][h]
    float2* V;          // [l][r][h]
    float* inv_sigma;   // [r][h] (0 below the rank tolerance)
    float* feat;        // [r][h][4]: |n| / (2T), log10 sigma, (unused), layer weight
    float* s;           // [l][h] layer scale gamma^(1/2) / c (1 + tau |n|^2)^(-beta/2)
    float2* ph;         // [g][l][h] forward-operator phases exp(2 pi i n . s_gl / M)
    float* mult;        // [h] half-spectrum multiplicity (2, 1, or 0 on Nyquist)
};

struct LearnSetupArgs {
    int M, G, L, r;
    double T, beta;
    double c[kMaxL], sqrt_gamma[kMaxL], gamma[kMaxL];
    double sx[kMaxG * kMaxL], sy[kMaxG * kMaxL];   // layer-pixel shifts [g * kMaxL + l]
    const double2* W;
    const double2* Q;
    const double* sigma;
    LearnFreq* freq;                                 // device copy of the pointers
};

struct LearnStatsArgs {
    const LearnFreq* freq;
    const float* amp;         // [l][h]
    const float2* zl;         // [f][l][h]
    const float2* zn;         // [f][g][h]
    const float* eta;         // [f] (device)
    float* stats;             // [frame][h][stride]: Q (r x r), c (r), |F|^2
    float noise_scale;        // sigma_n M per unit eta
    int G, L, r, count, first, stride;
    size_t H;
};

struct MlpRowsArgs {
    const float* params;
    const float* feat;        // LearnFreq::feat
    const float* mult;
    const float* stats;
    const float* eta;         // per stored frame
    const int* frames;        // [nb] frame indices
    float* act;               // [ACT_PLANES][rows]
    float* loss_part;         // [blocks]
    float scale;              // 1 / (Z nb)
    int nb, r, stride;
    size_t H;
};

struct MlpGradArgs {
    const float* act;
    float* partials;          // [chunks][8705]
    size_t rows, rows_per_chunk;
};

struct MlpAdamArgs {
    const float* partials;
    int chunks;
    float* grad_out;          // optional
    int update;
    float* params;
    float* m;
    float* v;
    float lr, b1, b2, eps, b1t, b2t;
};

// Filter factors evaluated against the stored statistics of a set of frames, one thread per frequency h:
// Qbar, cbar, |F|^2 summed over the frames (FP64), then either the optimum phi* = Qbar^-1 cbar over the
// components above the cutoff (mode 0) or Tikhonov's phi = sigma^2 / (sigma^2 + alpha) (mode 1);
// loss[h] = mult_h (phi^T Qbar phi - 2 cbar^T phi + |F|^2).
struct FilterEvalArgs {
    const LearnFreq* freq;
    const float* stats;       // [frame][h][stride]
    const int* frames;        // [nb]
    float* phi;               // [r][h] (mode 0 output, or nullptr)
    double* loss;             // [h]
    double alpha;             // mode 1
    int nb, r, stride, mode;
    size_t H;
};

__global__ void learn_setup_kernel(LearnSetupArgs a);
__global__ void filter_eval_kernel(FilterEvalArgs a);
__global__ void learn_stats_kernel(LearnStatsArgs a);
__global__ void mlp_rows_kernel(MlpRowsArgs a);
__global__ void mlp_wgrad_kernel(MlpGradArgs a);
__global__ void mlp_adam_kernel(MlpAdamArgs a);
size_t mlp_rows_lds_bytes(int threads);

}  // namespace safr
