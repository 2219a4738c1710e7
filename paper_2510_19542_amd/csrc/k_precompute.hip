// Soft-real-time precomputation of B (Alg. 2) in FP64, one thread per
// half-spectrum frequency (j, k), k = 0..M/2.
//
// svd_kernel: builds the G x L matrix A_n of Sec. 3.1,
//     A[g, l] = s_l(n) exp(i pi h_l (n_x ax_g + n_y ay_g) / (c_l T)),
//     s_l(n) = gamma_l^(1/2) / c_l (1 + pi^2 |n|^2 / (c_l T)^2)^(-beta/2),
//   and orthogonalises the columns of X = A (L <= G) or X = A^H (G < L) by
//   one-sided (Hestenes) complex Jacobi rotations: X Q = W with orthogonal
//   columns, sigma_c = |W_c|.
// assemble_kernel: B_n[l, g] = s_l(n) sum_r V[l, r] g(sigma_r) conj(U[g, r]),
//   which in terms of W and Q is
//     L <= G (U = W / sigma, V = Q):   s_l sum_c Q[l, c] h_c conj(W[g, c]),
//     G <  L (U = Q, V = W / sigma):   s_l sum_c W[l, c] h_c conj(Q[g, c]),
//   with h_c = g(sigma_c) / sigma_c: Tikhonov 1 / (sigma^2 + alpha); alpha = 0
//   gives 1 / sigma^2 above the rank tolerance max(G, L) eps sigma_1; the learned
//   filter gives phi_c / sigma^2 above sqrt(eps) sigma_1 (a factor phi in (0, 1)
//   does not vanish as sigma -> 0, so rounding-level singular values of exactly
//   rank-deficient frequencies would otherwise become gains of order 1 / eps).
// The k = 0 column is mirrored (B(-j, 0) = conj B(j, 0)) so that B is exactly
// Hermitian, and the Nyquist row and column are zero.
#include <cmath>

#include "safr_internal.h"

namespace safr {

namespace {

struct Z { double x, y; };
__device__ __forceinline__ Z zmul(Z a, Z b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ Z zconj(Z a) { return {a.x, -a.y}; }
__device__ __forceinline__ double zabs2(Z a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ int shifted(int j, int M) { return j <= (M - 1) / 2 ? j : j - M; }

__device__ __forceinline__ double layer_scale(const PrecompArgs& a, int l, double nx, double ny) {
    const double ct = a.c[l] * a.T;
    const double tau = M_PI * M_PI / (ct * ct);
    return a.sqrt_gamma[l] / a.c[l] * pow(1.0 + tau * (nx * nx + ny * ny), -0.5 * a.beta);
}

}  // namespace

__global__ void svd_kernel(PrecompArgs a) {
    const int M = a.M, G = a.G, L = a.L;
    const int Kh = M / 2 + 1;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= Kh * M) return;
    const int k = h / M, j = h % M;
    const bool flip = G < L;
    const int R = flip ? L : G, C = flip ? G : L;
    const int nx = shifted(j, M), ny = shifted(k, M);

    Z X[kMaxG * kMaxL];
    Z Q[kMaxL * kMaxL];
    for (int g = 0; g < G; ++g) {
        for (int l = 0; l < L; ++l) {
            const double s = layer_scale(a, l, nx, ny);
            double sn, cs;
            sincospi(a.h[l] * (nx * a.ax[g] + ny * a.ay[g]) / (a.c[l] * a.T), &sn, &cs);
            const Z v = {s * cs, s * sn};
            if (flip) X[l * C + g] = zconj(v);
            else X[g * C + l] = v;
        }
    }
    for (int p = 0; p < C; ++p)
        for (int q = 0; q < C; ++q) Q[p * C + q] = {p == q ? 1.0 : 0.0, 0.0};
    // pairs whose inner product is negligible against the whole matrix are left alone, so
    // numerically zero columns of a rank-deficient A (the zero frequency) stop rotating
    double fro = 0.0;
    for (int i = 0; i < R * C; ++i) fro += zabs2(X[i]);
    const double floor_ = 1e-30 * fro;

    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < C - 1; ++p) {
            for (int q = p + 1; q < C; ++q) {
                double aa = 0.0, bb = 0.0;
                Z cc = {0.0, 0.0};
                for (int r = 0; r < R; ++r) {
                    const Z xp = X[r * C + p], xq = X[r * C + q];
                    aa += zabs2(xp);
                    bb += zabs2(xq);
                    cc = {cc.x + xp.x * xq.x + xp.y * xq.y, cc.y + xp.x * xq.y - xp.y * xq.x};
                }
                const double mag = sqrt(zabs2(cc));
                if (!(mag > 1e-15 * sqrt(aa * bb)) || !(mag > floor_)) continue;
                rotated = true;
                const Z e = {cc.x / mag, -cc.y / mag};           // exp(-i theta)
                const double zeta = (bb - aa) / (2.0 * mag);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t);
                const double sn = t * cs;
                for (int r = 0; r < R; ++r) {
                    const Z xp = X[r * C + p];
                    const Z exq = zmul(e, X[r * C + q]);
                    X[r * C + p] = {cs * xp.x - sn * exq.x, cs * xp.y - sn * exq.y};
                    X[r * C + q] = {sn * xp.x + cs * exq.x, sn * xp.y + cs * exq.y};
                }
                for (int r = 0; r < C; ++r) {
                    const Z xp = Q[r * C + p];
                    const Z exq = zmul(e, Q[r * C + q]);
                    Q[r * C + p] = {cs * xp.x - sn * exq.x, cs * xp.y - sn * exq.y};
                    Q[r * C + q] = {sn * xp.x + cs * exq.x, sn * xp.y + cs * exq.y};
                }
            }
        }
        if (!rotated) break;
    }

    double2* W = a.W + (size_t)h * R * C;
    double2* Qo = a.Q + (size_t)h * C * C;
    for (int i = 0; i < R * C; ++i) W[i] = make_double2(X[i].x, X[i].y);
    for (int i = 0; i < C * C; ++i) Qo[i] = make_double2(Q[i].x, Q[i].y);
    for (int c = 0; c < C; ++c) {
        double s2 = 0.0;
        for (int r = 0; r < R; ++r) s2 += zabs2(X[r * C + c]);
        const double sig = sqrt(s2);
        a.sigma[(size_t)h * C + c] = sig;
        if (a.feats) {
            double w = 0.0;
            if (flip) {
                for (int l = 0; l < L; ++l) w += a.gamma[l] * zabs2(X[l * C + c]);
                w = sig > 0.0 ? w / s2 : 0.0;
            } else {
                for (int l = 0; l < L; ++l) w += a.gamma[l] * zabs2(Q[l * C + c]);
            }
            float* fo = a.feats + ((size_t)h * C + c) * 4;
            fo[0] = (float)(sqrt((double)nx * nx + (double)ny * ny) / (2.0 * a.T));
            fo[1] = (float)log10(fmax(sig, 1e-30));
            fo[2] = (float)a.log10_noise;
            fo[3] = (float)w;
        }
    }
}

__global__ void assemble_kernel(PrecompArgs a) {
    const int M = a.M, G = a.G, L = a.L;
    const int Kh = M / 2 + 1;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= Kh * M) return;
    const int k = h / M, j = h % M;
    const bool flip = G < L;
    const int R = flip ? L : G, C = flip ? G : L;
    const bool nyq = (M % 2 == 0) && (j == M / 2 || k == M / 2);
    const bool mirror = (k == 0) && (j > M / 2);
    const int js = mirror ? M - j : j;                  // frequency whose SVD is used
    const int hs = k * M + js;
    const int nx = shifted(js, M), ny = shifted(k, M);

    const double2* W = a.W + (size_t)hs * R * C;
    const double2* Qm = a.Q + (size_t)hs * C * C;
    const double* sg = a.sigma + (size_t)hs * C;
    double smax = 0.0;
    for (int c = 0; c < C; ++c) smax = fmax(smax, sg[c]);
    const double tol = (double)(G > L ? G : L) * 2.220446049250313e-16 * smax;
    // regularisation parameter of this frequency (the weight map is point-symmetric, so the mirrored
    // frequency's value is the same)
    const double an = a.aw ? a.alpha * a.aw[(size_t)js * M + k] : a.alpha;
    double hv[kMaxL];
    for (int c = 0; c < C; ++c) {
        const double s = sg[c];
        double v;
        if (a.phi) v = s > kSqrtEps * smax ? (double)a.phi[(size_t)hs * C + c] / (s * s) : 0.0;
        else if (a.tsvd) v = (s > tol && s * s > an) ? 1.0 / (s * s) : 0.0;
        else if (an > 0.0) v = 1.0 / (s * s + an);
        else v = s > tol ? 1.0 / (s * s) : 0.0;
        hv[c] = v;
    }
    bool bad = false;
    for (int l = 0; l < L; ++l) {
        const double sl = layer_scale(a, l, nx, ny);
        for (int g = 0; g < G; ++g) {
            Z acc = {0.0, 0.0};
            for (int c = 0; c < C; ++c) {
                Z lhs, rhs;
                if (flip) {
                    lhs = {W[l * C + c].x, W[l * C + c].y};
                    rhs = {Qm[g * C + c].x, -Qm[g * C + c].y};
                } else {
                    lhs = {Qm[l * C + c].x, Qm[l * C + c].y};
                    rhs = {W[g * C + c].x, -W[g * C + c].y};
                }
                const Z p = zmul(lhs, rhs);
                acc.x += hv[c] * p.x;
                acc.y += hv[c] * p.y;
            }
            Z b = {sl * acc.x, sl * acc.y};
            if (mirror) b.y = -b.y;
            if (nyq) b = {0.0, 0.0};
            if (!isfinite(b.x) || !isfinite(b.y)) bad = true;
            const size_t o = (((size_t)k * L + l) * G + g) * M + j;
            a.B64[o] = make_double2(b.x, b.y);
            // FP32 copy in the column-pass layout: [k / CPW][l][g][k % CPW][j], CPW = 256 / M, with the
            // 1/M^2 of IDFT2 folded in (M^2 is a power of two, so the scaling is exact)
            const int cpw = 256 / M;
            const size_t o32 = ((((size_t)(k / cpw) * L + l) * G + g) * cpw + (k % cpw)) * M + j;
            const double inv_m2 = 1.0 / ((double)M * (double)M);
            a.B32[o32] = make_float2((float)(b.x * inv_m2), (float)(b.y * inv_m2));
        }
    }
    if (bad) atomicOr(a.bad, 1);
}

hipError_t launch_svd(const PrecompArgs& a, hipStream_t s) {
    const int H = (a.M / 2 + 1) * a.M;
    hipLaunchKernelGGL(svd_kernel, dim3((H + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_assemble(const PrecompArgs& a, hipStream_t s) {
    const int H = (a.M / 2 + 1) * a.M;
    hipLaunchKernelGGL(assemble_kernel, dim3((H + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace safr
