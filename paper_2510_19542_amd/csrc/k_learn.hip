// Learned spectral filter: the network that replaces Tikhonov's filter factors
// (Sec. 3.1 admits any regularising filter g; here g_r = phi_r / sigma_r with
// phi = MLP(|n| / (2T), log10 sigma_r, log10 eta, sum_l gamma_l |V_lr|^2)).
//
// Network 4 -> 64 -> 64 -> 64 -> 1, exact GELU x Phi(x) after each hidden layer,
// logistic output.  Flat parameters: W1 (64 x 4), b1, W2 (64 x 64), b2, W3, b3,
// w4 (64), b4 (8,705 floats; W[out][in]).
//
// Training data (periodic-exact mode): layer spectra F_l = amp_l z_l, wavefront
// spectra d_g = sum_l exp(2 pi i n . s_gl / M) F_l + eta sigma_n M z_g (the
// tomography operator in Fourier form), and per frequency the statistics of the
// layer residual, which is quadratic in phi:
//   |b - F|^2 = phi^T Q phi - 2 c^T phi + |F|^2,  y = U^H d,
//   Q_rq = Re(conj(y_r) y_q sum_l s_l^2 conj(V_lr) V_lq) / (sigma_r sigma_q),
//   c_r  = Re(y_r sum_l conj(F_l) s_l V_lr) / sigma_r.
// Training (FP32): row kernel (forward, dL/dphi, backward to the pre-activation
// gradients, one thread per frame and frequency, weights in LDS), weight-gradient
// tiles (outer products summed over rows), Adam (Kingma & Ba 2015).
// Inference for the precompute: BF16 inputs and weights on matrix cores
// (v_mfma_f32_16x16x32_bf16) for the two 64 x 64 layers, FP32 accumulation.
#include <cmath>

#include "learn_internal.h"

namespace safr {

namespace {

constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 320, OFF_B2 = 4416, OFF_W3 = 4480, OFF_B3 = 8576,
              OFF_W4 = 8640, OFF_B4 = 8704;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

struct Zd {
    double x, y;
};
__device__ __forceinline__ Zd zd(double2 v) { return {v.x, v.y}; }

}  // namespace

// ----------------------------------------------------------------------------------------
// Per-frequency constants for training: U, V (normalised), sigma, rank mask, layer scale,
// forward-operator phases, multiplicity, features (f0, log10 sigma, -, layer weight).
// ----------------------------------------------------------------------------------------
__global__ void learn_setup_kernel(LearnSetupArgs a) {
    const int M = a.M, G = a.G, L = a.L, r = a.r, Kh = M / 2 + 1;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= Kh * M) return;
    const int k = h / M, j = h % M;
    const int nx = j <= (M - 1) / 2 ? j : j - M, ny = k <= (M - 1) / 2 ? k : k - M;
    const bool flip = G < L;
    const int R = flip ? L : G, C = flip ? G : L;       // C == r
    const double2* W = a.W + (size_t)h * R * C;
    const double2* Q = a.Q + (size_t)h * C * C;
    const double* sg = a.sigma + (size_t)h * C;
    double smax = 0.0;
    for (int c = 0; c < C; ++c) smax = fmax(smax, sg[c]);
    const double tol = kSqrtEps * smax;                 // the learned filter's cutoff
    LearnFreq* fq = a.freq;
    const size_t H = (size_t)Kh * M;
    for (int c = 0; c < r; ++c) {
        const double s = sg[c];
        const bool ok = s > tol;
        const double inv = ok ? 1.0 / s : 0.0;
        for (int g = 0; g < G; ++g) {
            // U[g][c]
            const Zd u = flip ? zd(Q[g * C + c]) : Zd{W[g * C + c].x * inv, W[g * C + c].y * inv};
            fq->U[((size_t)g * r + c) * H + h] = make_float2((float)u.x, (float)u.y);
        }
        double wl = 0.0;
        for (int l = 0; l < L; ++l) {
            const Zd v = flip ? Zd{W[l * C + c].x * inv, W[l * C + c].y * inv} : zd(Q[l * C + c]);
            fq->V[((size_t)l * r + c) * H + h] = make_float2((float)v.x, (float)v.y);
            wl += a.gamma[l] * (v.x * v.x + v.y * v.y);
        }
        fq->inv_sigma[(size_t)c * H + h] = (float)inv;
        float* ft = fq->feat + ((size_t)c * H + h) * 4;
        ft[0] = (float)(sqrt((double)nx * nx + (double)ny * ny) / (2.0 * a.T));
        ft[1] = (float)log10(fmax(s, 1e-30));
        ft[2] = 0.f;
        ft[3] = ok ? (float)wl : 0.f;
    }
    for (int l = 0; l < L; ++l) {
        const double ct = a.c[l] * a.T;
        fq->s[(size_t)l * H + h] = (float)(a.sqrt_gamma[l] / a.c[l] *
                                           pow(1.0 + M_PI * M_PI / (ct * ct) * (nx * nx + ny * ny), -0.5 * a.beta));
        for (int g = 0; g < G; ++g) {
            double sn, cs;
            sincospi(2.0 * (nx * a.sx[g * kMaxL + l] + ny * a.sy[g * kMaxL + l]) / M, &sn, &cs);
            fq->ph[((size_t)g * L + l) * H + h] = make_float2((float)cs, (float)sn);
        }
    }
    const bool nyq = (M % 2 == 0) && (j == M / 2 || k == M / 2);
    fq->mult[h] = nyq ? 0.f : (k == 0 ? 1.f : 2.f);
}

// ----------------------------------------------------------------------------------------
// Filter factors against the training objective (see FilterEvalArgs).  The objective is quadratic in phi
// at every frequency, so its minimum over all filter factors (any network's, Tikhonov's, ...) is reached
// at phi* = Qbar^-1 cbar, solved here by Gaussian elimination with partial pivoting over the components
// above the cutoff (the others carry Q = c = 0 and get phi = 0).
// ----------------------------------------------------------------------------------------
__global__ void filter_eval_kernel(FilterEvalArgs a) {
    const size_t h = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= a.H) return;
    const int r = a.r;
    const LearnFreq& fq = *a.freq;
    double Q[kMaxG][kMaxG], c[kMaxG], phi[kMaxG];
    double f2 = 0.0;
    for (int i = 0; i < r; ++i) {
        c[i] = 0.0;
        for (int q = 0; q < r; ++q) Q[i][q] = 0.0;
    }
    for (int b = 0; b < a.nb; ++b) {
        const float* st = a.stats + ((size_t)a.frames[b] * a.H + h) * a.stride;
        for (int i = 0; i < r; ++i) {
            for (int q = 0; q < r; ++q) Q[i][q] += st[i * r + q];
            c[i] += st[r * r + i];
        }
        f2 += st[r * r + r];
    }
    bool ok[kMaxG];
    for (int i = 0; i < r; ++i) ok[i] = fq.inv_sigma[(size_t)i * a.H + h] > 0.f;
    if (a.mode == 0) {
        // solve over the kept components (the rest: phi = 0); A = Q restricted, x = c restricted
        int idx[kMaxG], n = 0;
        for (int i = 0; i < r; ++i)
            if (ok[i]) idx[n++] = i;
        double A[kMaxG][kMaxG + 1];
        for (int i = 0; i < n; ++i) {
            for (int q = 0; q < n; ++q) A[i][q] = Q[idx[i]][idx[q]];
            A[i][n] = c[idx[i]];
        }
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int i = col + 1; i < n; ++i)
                if (fabs(A[i][col]) > fabs(A[piv][col])) piv = i;
            if (piv != col)
                for (int q = 0; q <= n; ++q) {
                    const double tmp = A[col][q];
                    A[col][q] = A[piv][q];
                    A[piv][q] = tmp;
                }
            const double d = A[col][col];
            for (int i = col + 1; i < n; ++i) {
                const double m = d != 0.0 ? A[i][col] / d : 0.0;
                for (int q = col; q <= n; ++q) A[i][q] -= m * A[col][q];
            }
        }
        double x[kMaxG];
        for (int i = n - 1; i >= 0; --i) {
            double acc = A[i][n];
            for (int q = i + 1; q < n; ++q) acc -= A[i][q] * x[q];
            x[i] = A[i][i] != 0.0 ? acc / A[i][i] : 0.0;
        }
        for (int i = 0; i < r; ++i) phi[i] = 0.0;
        for (int i = 0; i < n; ++i) phi[idx[i]] = x[i];
        if (a.phi)
            for (int i = 0; i < r; ++i) a.phi[(size_t)i * a.H + h] = (float)phi[i];
    } else {
        for (int i = 0; i < r; ++i) {
            const double inv = fq.inv_sigma[(size_t)i * a.H + h];
            const double s2 = inv > 0.0 ? 1.0 / (inv * inv) : 0.0;
            phi[i] = ok[i] ? s2 / (s2 + a.alpha) : 0.0;
        }
    }
    double quad = f2;
    for (int i = 0; i < r; ++i) {
        double qp = 0.0;
        for (int q = 0; q < r; ++q) qp += Q[i][q] * phi[q];
        quad += phi[i] * qp - 2.0 * c[i] * phi[i];
    }
    a.loss[h] = (double)fq.mult[h] * quad;
}

// ----------------------------------------------------------------------------------------
// Statistics (Q, c, |F|^2) of frames f0 .. f0+count-1, one thread per (frame, frequency).
// ----------------------------------------------------------------------------------------
__global__ void learn_stats_kernel(LearnStatsArgs a) {
    const int G = a.G, L = a.L, r = a.r;
    const size_t H = a.H;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)a.count * H) return;
    const int f = (int)(e / H);
    const size_t h = e % H;
    const LearnFreq& fq = *a.freq;
    const float eta = a.eta[f];
    float2 F[kMaxL], D[kMaxG];
    float f2 = 0.f;
    for (int l = 0; l < L; ++l) {
        const float am = a.amp[(size_t)l * H + h];
        const float2 z = a.zl[((size_t)f * L + l) * H + h];
        F[l] = make_float2(am * z.x, am * z.y);
        f2 += F[l].x * F[l].x + F[l].y * F[l].y;
    }
    const float ns = eta * a.noise_scale;
    for (int g = 0; g < G; ++g) {
        const float2 z = a.zn[((size_t)f * G + g) * H + h];
        float2 acc = make_float2(ns * z.x, ns * z.y);
        for (int l = 0; l < L; ++l) {
            const float2 p = fq.ph[((size_t)g * L + l) * H + h];
            acc.x += p.x * F[l].x - p.y * F[l].y;
            acc.y += p.x * F[l].y + p.y * F[l].x;
        }
        D[g] = acc;
    }
    float2 y[kMaxL];
    float inv[kMaxL];
    for (int c = 0; c < r; ++c) {
        float2 acc = make_float2(0.f, 0.f);
        for (int g = 0; g < G; ++g) {
            const float2 u = fq.U[((size_t)g * r + c) * H + h];
            acc.x += u.x * D[g].x + u.y * D[g].y;          // conj(u) d
            acc.y += u.x * D[g].y - u.y * D[g].x;
        }
        y[c] = acc;
        inv[c] = fq.inv_sigma[(size_t)c * H + h];
    }
    float* out = a.stats + ((size_t)(a.first + f) * H + h) * a.stride;
    for (int c = 0; c < r; ++c) {
        for (int q = 0; q < r; ++q) {
            // sum_l s_l^2 conj(V_lc) V_lq
            float wr = 0.f, wi = 0.f;
            for (int l = 0; l < L; ++l) {
                const float sl = fq.s[(size_t)l * H + h];
                const float2 vc = fq.V[((size_t)l * r + c) * H + h], vq = fq.V[((size_t)l * r + q) * H + h];
                wr += sl * sl * (vc.x * vq.x + vc.y * vq.y);
                wi += sl * sl * (vc.x * vq.y - vc.y * vq.x);
            }
            // Re(conj(y_c) y_q (wr + i wi))
            const float pr = y[c].x * y[q].x + y[c].y * y[q].y;
            const float pi = y[c].x * y[q].y - y[c].y * y[q].x;
            out[c * r + q] = (pr * wr - pi * wi) * inv[c] * inv[q];
        }
        float tr = 0.f, ti = 0.f;                          // sum_l conj(F_l) s_l V_lc
        for (int l = 0; l < L; ++l) {
            const float sl = fq.s[(size_t)l * H + h];
            const float2 v = fq.V[((size_t)l * r + c) * H + h];
            tr += sl * (F[l].x * v.x + F[l].y * v.y);
            ti += sl * (F[l].x * v.y - F[l].y * v.x);
        }
        out[r * r + c] = (y[c].x * tr - y[c].y * ti) * inv[c];
    }
    out[r * r + r] = f2;
}

// ----------------------------------------------------------------------------------------
// Training row kernel: thread per (batch frame b, frequency h), rows c < r.
// Activation store layout: act[v][i][row] (row fastest), rows = nb * H * r.
// ----------------------------------------------------------------------------------------
namespace {

// LDS weight layout (floats): W1[256] b1[64] W2[4096] b2[64] W3[4096] b3[64] w4[64] b4[1] | W2T[4096] W3T[4096]
constexpr int LDS_W = 8705, LDS_W2T = 8708, LDS_W3T = LDS_W2T + 4096, LDS_PARAMS = LDS_W3T + 4096;

__device__ __forceinline__ void load_weights(const float* __restrict__ p, float* w) {
    for (int i = threadIdx.x; i < LDS_W; i += blockDim.x) w[i] = p[i];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) {
        const int o = i / 64, c = i % 64;
        w[LDS_W2T + c * 64 + o] = p[OFF_W2 + i];
        w[LDS_W3T + c * 64 + o] = p[OFF_W3 + i];
    }
}

// out[o] = act(sum_i Wrow[o][i] x[i] + b[o]) for o < 64; x in registers; each output is
// written to the thread's LDS slot (slot[o * nthr]) and to the global planes (a, g).
__device__ __forceinline__ void dense64(const float* w, const float* b, const float (&x)[64], float* slot, int nthr,
                                        float* ga, float* gg, size_t plane, size_t row) {
    for (int o = 0; o < 64; ++o) {
        const float4* wr = reinterpret_cast<const float4*>(w + o * 64);
        float acc = b[o];
#pragma unroll
        for (int i4 = 0; i4 < 16; ++i4) {
            const float4 v = wr[i4];
            acc += v.x * x[4 * i4] + v.y * x[4 * i4 + 1] + v.z * x[4 * i4 + 2] + v.w * x[4 * i4 + 3];
        }
        const float av = gelu(acc);
        slot[o * nthr] = av;
        ga[(size_t)o * plane + row] = av;
        gg[(size_t)o * plane + row] = gelu_grad(acc);
    }
}

}  // namespace

__global__ __launch_bounds__(128) void mlp_rows_kernel(MlpRowsArgs a) {
    extern __shared__ float lds[];
    float* w = lds;
    float* slots = lds + LDS_PARAMS;
    const int nthr = blockDim.x;
    float* slot = slots + threadIdx.x;
    load_weights(a.params, w);
    __syncthreads();
    const int r = a.r;
    const size_t H = a.H;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = e < (size_t)a.nb * H;
    const int b = live ? (int)(e / H) : 0;
    const size_t h = live ? e % H : 0;
    const int frame = live ? a.frames[b] : 0;
    const size_t plane = (size_t)a.nb * H * r;
    float phi[kMaxL];
    float loss = 0.f;
    if (live) {
        const float lg_eta = log10f(a.eta[frame]);
        // forward every row of this frequency
        for (int c = 0; c < r; ++c) {
            const size_t row = (e * r) + c;
            const float* ft = a.feat + ((size_t)c * H + h) * 4;
            const float xin[4] = {ft[0], ft[1], lg_eta, ft[3]};
            float x[64];
#pragma unroll
            for (int i = 0; i < 4; ++i) a.act[(size_t)(ACT_X + i) * plane + row] = xin[i];
            for (int o = 0; o < 64; ++o) {
                const float z = w[OFF_B1 + o] + w[OFF_W1 + 4 * o] * xin[0] + w[OFF_W1 + 4 * o + 1] * xin[1] +
                                w[OFF_W1 + 4 * o + 2] * xin[2] + w[OFF_W1 + 4 * o + 3] * xin[3];
                const float av = gelu(z);
                slot[o * nthr] = av;
                a.act[((size_t)ACT_A1 + o) * plane + row] = av;
                a.act[((size_t)ACT_G1 + o) * plane + row] = gelu_grad(z);
            }
#pragma unroll
            for (int i = 0; i < 64; ++i) x[i] = slot[i * nthr];
            dense64(w + OFF_W2, w + OFF_B2, x, slot, nthr, a.act + (size_t)ACT_A2 * plane, a.act + (size_t)ACT_G2 * plane,
                    plane, row);
#pragma unroll
            for (int i = 0; i < 64; ++i) x[i] = slot[i * nthr];
            dense64(w + OFF_W3, w + OFF_B3, x, slot, nthr, a.act + (size_t)ACT_A3 * plane, a.act + (size_t)ACT_G3 * plane,
                    plane, row);
            float z4 = w[OFF_B4];
            for (int i = 0; i < 64; ++i) z4 += w[OFF_W4 + i] * slot[i * nthr];
            phi[c] = sigmoid(z4);
        }
        // dL/dphi = 2 m (Q phi - c) / (Z nb); loss = m (phi Q phi - 2 c phi + |F|^2) / (Z nb)
        const float* st = a.stats + ((size_t)frame * H + h) * a.stride;
        const float m = a.mult[h] * a.scale;
        float dphi[kMaxL];
        for (int c = 0; c < r; ++c) {
            float qp = 0.f;
            for (int q = 0; q < r; ++q) qp += st[c * r + q] * phi[q];
            dphi[c] = 2.f * m * (qp - st[r * r + c]);
            loss += m * (phi[c] * qp - 2.f * st[r * r + c] * phi[c]);
        }
        loss += m * st[r * r + r];
        // backward every row
        for (int c = 0; c < r; ++c) {
            const size_t row = (e * r) + c;
            const float dz4 = dphi[c] * phi[c] * (1.f - phi[c]);
            a.act[(size_t)ACT_DZ4 * plane + row] = dz4;
            float d[64];
#pragma unroll
            for (int i = 0; i < 64; ++i) {
                d[i] = dz4 * w[OFF_W4 + i] * a.act[((size_t)ACT_G3 + i) * plane + row];
                a.act[((size_t)ACT_DZ3 + i) * plane + row] = d[i];
            }
            // dz2 = (W3^T dz3) * gelu'(z2)
            for (int i = 0; i < 64; ++i) {
                const float4* wr = reinterpret_cast<const float4*>(w + LDS_W3T + i * 64);
                float acc = 0.f;
#pragma unroll
                for (int o4 = 0; o4 < 16; ++o4) {
                    const float4 v = wr[o4];
                    acc += v.x * d[4 * o4] + v.y * d[4 * o4 + 1] + v.z * d[4 * o4 + 2] + v.w * d[4 * o4 + 3];
                }
                const float dz = acc * a.act[((size_t)ACT_G2 + i) * plane + row];
                slot[i * nthr] = dz;
                a.act[((size_t)ACT_DZ2 + i) * plane + row] = dz;
            }
#pragma unroll
            for (int i = 0; i < 64; ++i) d[i] = slot[i * nthr];
            // dz1 = (W2^T dz2) * gelu'(z1)
            for (int i = 0; i < 64; ++i) {
                const float4* wr = reinterpret_cast<const float4*>(w + LDS_W2T + i * 64);
                float acc = 0.f;
#pragma unroll
                for (int o4 = 0; o4 < 16; ++o4) {
                    const float4 v = wr[o4];
                    acc += v.x * d[4 * o4] + v.y * d[4 * o4 + 1] + v.z * d[4 * o4 + 2] + v.w * d[4 * o4 + 3];
                }
                a.act[((size_t)ACT_DZ1 + i) * plane + row] = acc * a.act[((size_t)ACT_G1 + i) * plane + row];
            }
        }
    }
    // per-block loss partial
    __shared__ float red[4];
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < (nthr + 63) / 64; ++i) s += red[i];
        a.loss_part[blockIdx.x] = s;
    }
}

size_t mlp_rows_lds_bytes(int threads) { return (size_t)(LDS_PARAMS + 64 * threads) * sizeof(float); }

// ----------------------------------------------------------------------------------------
// Weight gradients: sum over rows of dz (outputs) x a (inputs); partials per row chunk.
// blockIdx.y selects layer 1 (64 x 4), 2 (64 x 64), 3 (64 x 64), 4 (1 x 64); biases too.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(MlpGradArgs a) {
    constexpr int RB = 32;                                  // rows staged per round
    __shared__ float sdz[RB][65];
    __shared__ float sa[RB][65];
    const int layer = blockIdx.y + 1;
    const size_t plane = a.rows;
    const size_t r0 = (size_t)blockIdx.x * a.rows_per_chunk;
    const size_t r1 = min(a.rows, r0 + a.rows_per_chunk);
    const int O = layer == 4 ? 1 : 64, I = layer == 1 ? 4 : 64;
    const int dzv = layer == 1 ? ACT_DZ1 : layer == 2 ? ACT_DZ2 : layer == 3 ? ACT_DZ3 : ACT_DZ4;
    const int av = layer == 1 ? ACT_X : layer == 2 ? ACT_A1 : ACT_A2;
    const int av4 = ACT_A3;
    const int tid = threadIdx.x;
    // thread tile: 4 outputs x 4 inputs for the 64 x 64 layers; otherwise one (o, i) each
    const int to = tid / 16, ti = tid % 16;
    float acc[4][4] = {};
    float accb = 0.f;                                       // bias: sum of dz[o = tid]
    for (size_t base = r0; base < r1; base += RB) {
        const int nr = (int)min((size_t)RB, r1 - base);
        // stage dz[o][rows] and a[i][rows] as [row][o], [row][i]
        for (int idx = tid; idx < RB * O; idx += 256) {
            const int rr = idx % RB, o = idx / RB;
            sdz[rr][o] = rr < nr ? a.act[((size_t)dzv + o) * plane + base + rr] : 0.f;
        }
        const int II = layer == 4 ? 64 : I;
        const int avv = layer == 4 ? av4 : av;
        for (int idx = tid; idx < RB * II; idx += 256) {
            const int rr = idx % RB, i = idx / RB;
            sa[rr][i] = rr < nr ? a.act[((size_t)avv + i) * plane + base + rr] : 0.f;
        }
        __syncthreads();
        if (layer == 2 || layer == 3) {
            for (int rr = 0; rr < nr; ++rr) {
                float dv[4], xv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    dv[u] = sdz[rr][4 * to + u];
                    xv[u] = sa[rr][4 * ti + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += dv[u] * xv[v];
            }
        } else if (layer == 1) {
            if (tid < 256) {
                const int o = tid / 4, i = tid % 4;
                for (int rr = 0; rr < nr; ++rr) acc[0][0] += sdz[rr][o] * sa[rr][i];
            }
        } else {
            if (tid < 64)
                for (int rr = 0; rr < nr; ++rr) acc[0][0] += sdz[rr][0] * sa[rr][tid];
        }
        if (tid < O)
            for (int rr = 0; rr < nr; ++rr) accb += sdz[rr][tid];
        __syncthreads();
    }
    float* part = a.partials + (size_t)blockIdx.x * 8705;
    if (layer == 2 || layer == 3) {
        const int offw = layer == 2 ? OFF_W2 : OFF_W3;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[offw + (4 * to + u) * 64 + 4 * ti + v] = acc[u][v];
        if (tid < 64) part[(layer == 2 ? OFF_B2 : OFF_B3) + tid] = accb;
    } else if (layer == 1) {
        part[OFF_W1 + tid] = acc[0][0];                      // tid = o * 4 + i
        if (tid < 64) part[OFF_B1 + tid] = accb;
    } else {
        if (tid < 64) part[OFF_W4 + tid] = acc[0][0];
        if (tid == 0) part[OFF_B4] = accb;
    }
}

// Sum of the partial gradients, then one Adam step (Kingma & Ba 2015).
__global__ void mlp_adam_kernel(MlpAdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8705) return;
    float g = 0.f;
    for (int c = 0; c < a.chunks; ++c) g += a.partials[(size_t)c * 8705 + i];
    if (a.grad_out) a.grad_out[i] = g;
    if (!a.update) return;
    const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / (1.f - a.b1t), vh = v / (1.f - a.b2t);
    a.params[i] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

// ----------------------------------------------------------------------------------------
// BF16 inference on matrix cores: 16 rows per wavefront.
// ----------------------------------------------------------------------------------------
typedef __bf16 lbf16x8_t __attribute__((ext_vector_type(8)));
typedef float lf32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* __restrict__ params,
                                                        const float* __restrict__ feats, float* __restrict__ phi,
                                                        int rows, float log10_noise) {
    __shared__ float w[LDS_W];
    __shared__ float actx[4][64][17];                      // per wave: activations [feature][row] (padded)
    for (int i = threadIdx.x; i < LDS_W; i += blockDim.x) w[i] = params[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane / 16, rl = lane % 16;
    const int row = (blockIdx.x * 4 + wave) * 16 + rl;
    const bool live = row < rows;
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    if (live) {
        const float* f = feats + (size_t)row * 4;
        x[0] = f[0];
        x[1] = f[1];
        x[2] = log10_noise;
        x[3] = f[3];
    }
    auto r16 = [](float v) { return (float)(__bf16)v; };
    // layer 1 (VALU, bf16-rounded operands): lane group q computes the features 8q..8q+7 and 32+8q..
    float (*act)[17] = actx[wave];
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int o = 32 * half + 8 * q + v;
            float z = w[OFF_B1 + o];
#pragma unroll
            for (int i = 0; i < 4; ++i) z += r16(w[OFF_W1 + 4 * o + i]) * r16(x[i]);
            act[o][rl] = gelu(z);
        }
    __syncthreads();
    // layers 2 and 3 on matrix cores: D (64 outputs x 16 rows) = W (64 x 64) A (64 x 16 rows)
    for (int layer = 0; layer < 2; ++layer) {
        const int offw = layer == 0 ? OFF_W2 : OFF_W3, offb = layer == 0 ? OFF_B2 : OFF_B3;
        lbf16x8_t bop[2];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
#pragma unroll
            for (int v = 0; v < 8; ++v) bop[kc][v] = (__bf16)act[32 * kc + 8 * q + v][rl];
        lf32x4_t res[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            lf32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                lbf16x8_t aop;
#pragma unroll
                for (int v = 0; v < 8; ++v) aop[v] = (__bf16)w[offw + (16 * ot + rl) * 64 + 32 * kc + 8 * q + v];
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[kc], acc, 0, 0, 0);
            }
            res[ot] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * ot + 4 * q + v;
                act[o][rl] = gelu(res[ot][v] + w[offb + o]);
            }
        __syncthreads();
    }
    // layer 4: each lane group sums 16 of the 64 products, reduced over the four groups
    float z = 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = 16 * q + v;
        z += r16(w[OFF_W4 + i]) * r16(act[i][rl]);
    }
    z += __shfl_xor(z, 16, 64);
    z += __shfl_xor(z, 32, 64);
    if (live && q == 0) phi[row] = sigmoid(z + w[OFF_B4]);
}

hipError_t launch_mlp_infer(const float* params, const float* feats, float* phi, int rows, float log10_noise,
                            hipStream_t s) {
    const int blocks = (rows + 63) / 64;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3(blocks), dim3(256), 0, s, params, feats, phi, rows, log10_noise);
    return hipGetLastError();
}

}  // namespace safr
