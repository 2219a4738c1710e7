// Column pass of SAFR's hard-real-time step (Alg. 1), fused:
//   1. column FFT (length M) of each star's row spectrum R[.][k][.] (the input
//      is nonzero in the n pupil rows only, read directly from the row pass);
//   2. per-frequency apply b_l(j, k) = sum_g B[k][l][g][j] d_g(j, k) with the
//      group's FP32 B (Eq. sparseM: B is diagonal in frequency);
//   3. inverse column FFT of each layer spectrum, written as C[f][grp][l][k][p].
// The spectra d and b live only in LDS.  One block of 256 threads owns
// 256 / M columns of one group and loops over a chunk of frames.
//
// B is stored per block of columns as [l][g][column][j], so the block's whole
// B slice is one contiguous run and thread t owns the entries t, t + 256, ...
//
// Split tomography (Sec. 3.3): the least-squares plane b x + c y of each
// wavefront over the pupil is obtained from the moments written by the row
// pass; since the transform is linear, removing the plane (laser stars) is
// d_g -= b DFT2(x mask) + c DFT2(y mask) and keeping only the plane (natural
// stars) is d_g = b DFT2(x mask) + c DFT2(y mask), with the two transforms
// precomputed in FP64 per plan.
//
// Two kernels:
//   cols_fixed<M, L, G0, G1>: shapes known at compile time (the configured
//     geometries).  The block's B slice is loaded into registers once, right
//     after the first column-FFT inputs (loads retire in order, so the first
//     transform does not wait for B), and the apply is a branch-free unrolled
//     L x G product whose LDS reads issue together.
//   cols_generic<M>: any shape; B is read inside the apply loop.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

namespace {

struct ColGeom {
    int kb, k0, tid, team, t, c, j, k;
    bool kvalid;
    int f0, f1;
};

template <int M>
__device__ __forceinline__ ColGeom col_geom(const ColArgs& a) {
    using S = FftShape<M>;
    ColGeom q;
    q.kb = blockIdx.x;
    q.k0 = q.kb * (256 / M);
    q.tid = threadIdx.x;
    q.team = q.tid / S::T;
    q.t = q.tid % S::T;
    q.c = q.tid / M;
    q.j = q.tid % M;
    q.k = q.k0 + q.c;
    q.kvalid = q.k < M / 2 + 1;
    q.f0 = blockIdx.z * a.frames_per_block;
    q.f1 = min(a.frames, q.f0 + a.frames_per_block);
    return q;
}

// plane coefficients (b, c) of every star of the group for frame f, from the row-pass moments
__device__ __forceinline__ void plane_coefs(const ColArgs& a, const GroupArgs& gr, int G, int f, int tid,
                                            float2* coef) {
    if (tid < G) {
        const float* mo = a.mom + ((size_t)f * a.J + gr.star[tid]) * a.nchunk * 4;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
        for (int q = 0; q < a.nchunk; ++q) {
            m0 += mo[4 * q + 0];
            m1 += mo[4 * q + 1];
            m2 += mo[4 * q + 2];
        }
        coef[tid] = make_float2(a.tt_b[0] * m0 + a.tt_b[1] * m1 + a.tt_b[2] * m2,
                                a.tt_c[0] * m0 + a.tt_c[1] * m1 + a.tt_c[2] * m2);
    }
}

__device__ __forceinline__ float2 plane_value(float2 cf, float2 xh, float2 yh) {
    return make_float2(cf.x * xh.x + cf.y * yh.x, cf.x * xh.y + cf.y * yh.y);
}

// column-FFT inputs of task `task` (= column * G + member) for thread t: x[n1] = R[.][k][N2 n1 + t - p0]
template <int M>
__device__ __forceinline__ void load_column(const ColArgs& a, const GroupArgs& gr, int G, int ftasks, int k0,
                                            int f, int task, int t, float2 (&x)[FftShape<M>::N1]) {
    using S = FftShape<M>;
    const int cc = task / G, g = task - cc * G;
    const int kk = k0 + cc;
    if (task < ftasks && kk < M / 2 + 1) {
        const float2* col = a.R + (((size_t)f * a.J + gr.star[g]) * (M / 2 + 1) + kk) * a.n;
#pragma unroll
        for (int n1 = 0; n1 < S::N1; ++n1) {
            const int pr = S::N2 * n1 + t - a.p0;
            x[n1] = (pr >= 0 && pr < a.n) ? col[pr] : make_float2(0.f, 0.f);
        }
    }
}

// inverse column transforms of the L layer spectra in Bsp, written to C
template <int M>
__device__ __forceinline__ void inverse_columns(const ColArgs& a, const ColGeom& q, int gi, int L, int f,
                                                const float2* tws, float2* xch, const float2* Bsp) {
    constexpr int CPW = 256 / M, Kh = M / 2 + 1, NTEAM = 256 / FftShape<M>::T;
    const int itasks = CPW * L;
    for (int base = 0; base < itasks; base += NTEAM) {
        const int task = base + q.team;
        const int cc = task / L, l = task - cc * L;
        const int kk = q.k0 + cc;
        const bool active = task < itasks && kk < Kh;
        if (active) {
            const float2* src = Bsp + (cc * L + l) * M;
            fft_pass1<M, +1>(q.t, xch, tws, [&](int jj) -> float2 { return src[jj]; });
        }
        __syncthreads();
        if (active) {
            float2* dst = a.C + ((((size_t)f * a.groups.count + gi) * L + l) * Kh + kk) * M;
            fft_pass2<M, +1>(q.t, xch, [&](int p, float2 v) { dst[p] = v; });
        }
        __syncthreads();
    }
}

// LDS: tws[M] | xch[NTEAM][TL] | D[CPW][gmax][M] | Bsp[CPW][L][M] | coef[16]
template <int M>
__device__ __forceinline__ void carve(float2* smem, int gmax, int L, float2*& tws, float2*& xall, float2*& D,
                                      float2*& Bsp, float2*& coef) {
    constexpr int CPW = 256 / M, NTEAM = 256 / FftShape<M>::T;
    tws = smem;
    xall = tws + M;
    D = xall + NTEAM * team_lds<M>();
    Bsp = D + CPW * gmax * M;
    coef = Bsp + CPW * L * M;
}

template <int M, int L, int G, int MODE>
__device__ __forceinline__ void cols_body(const ColArgs& a, int gi, float2* smem) {
    using S = FftShape<M>;
    constexpr int CPW = 256 / M, NTEAM = 256 / S::T;
    constexpr int FT = MODE == 2 ? 0 : CPW * G;          // forward transforms per frame
    const GroupArgs& gr = a.groups.g[gi];
    const ColGeom q = col_geom<M>(a);
    float2 *tws, *xall, *D, *Bsp, *coef;
    carve<M>(smem, a.gmax, L, tws, xall, D, Bsp, coef);
    float2* xch = xall + q.team * team_lds<M>();

    // loads, oldest first: twiddles, first column inputs, B
    const float2 twv = q.tid < M ? a.tw[q.tid] : make_float2(0.f, 0.f);
    float2 x[S::N1];
    if constexpr (FT > 0) load_column<M>(a, gr, G, FT, q.k0, q.f0, q.team, q.t, x);
    const float2* Bblk = a.B + gr.b_off + (size_t)q.kb * L * G * 256;
    float2 breg[L * G];
#pragma unroll
    for (int i = 0; i < L * G; ++i) breg[i] = Bblk[(size_t)i * 256 + q.tid];
    float2 xh = make_float2(0.f, 0.f), yh = make_float2(0.f, 0.f);
    if (MODE != 0 && q.kvalid) {
        xh = a.Xh[(size_t)q.k * M + q.j];
        yh = a.Yh[(size_t)q.k * M + q.j];
    }
    if (q.tid < M) tws[q.tid] = twv;
    __syncthreads();

    for (int f = q.f0; f < q.f1; ++f) {
        if (MODE != 0) plane_coefs(a, gr, G, f, q.tid, coef);
        if constexpr (FT > 0) {
#pragma unroll
            for (int base = 0; base < FT; base += NTEAM) {
                const int task = base + q.team;
                const int cc = task / G, g = task - cc * G;
                const bool active = task < FT && q.k0 + cc < M / 2 + 1;
                if (f != q.f0 || base != 0) load_column<M>(a, gr, G, FT, q.k0, f, task, q.t, x);
                if (active) fft_pass1_regs<M, -1>(q.t, xch, tws, x);
                __syncthreads();
                if (active) {
                    float2* d = D + (cc * G + g) * M;
                    fft_pass2<M, -1>(q.t, xch, [&](int jj, float2 v) { d[jj] = v; });
                }
                __syncthreads();
            }
        } else {
            __syncthreads();
        }
        if (q.kvalid) {
            float2 dv[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if constexpr (MODE == 0) dv[g] = D[(q.c * G + g) * M + q.j];
                else if constexpr (MODE == 1) dv[g] = csub(D[(q.c * G + g) * M + q.j], plane_value(coef[g], xh, yh));
                else dv[g] = plane_value(coef[g], xh, yh);
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const float2 bv = breg[l * G + g];
                    acc.x += bv.x * dv[g].x - bv.y * dv[g].y;
                    acc.y += bv.x * dv[g].y + bv.y * dv[g].x;
                }
                Bsp[(q.c * L + l) * M + q.j] = acc;
            }
        }
        __syncthreads();
        inverse_columns<M>(a, q, gi, L, f, tws, xch, Bsp);
    }
}

}  // namespace

template <int M, int L, int G0, int G1>
__global__ __launch_bounds__(256, 2) void cols_fixed(ColArgs a) {
    extern __shared__ float2 smem[];
    if constexpr (G1 == 0) {
        cols_body<M, L, G0, 0>(a, 0, smem);
    } else {
        if (blockIdx.y == 0) cols_body<M, L, G0, 1>(a, 0, smem);
        else cols_body<M, L, G1, 2>(a, 1, smem);
    }
}

template <int M>
__global__ __launch_bounds__(256) void cols_generic(ColArgs a) {
    using S = FftShape<M>;
    constexpr int CPW = 256 / M, NTEAM = 256 / S::T;
    extern __shared__ float2 smem[];
    const int gi = blockIdx.y;
    const GroupArgs& gr = a.groups.g[gi];
    const int G = gr.G, mode = gr.mode, L = a.L;
    const ColGeom q = col_geom<M>(a);
    float2 *tws, *xall, *D, *Bsp, *coef;
    carve<M>(smem, a.gmax, L, tws, xall, D, Bsp, coef);
    float2* xch = xall + q.team * team_lds<M>();
    const int ftasks = mode == 2 ? 0 : CPW * G;
    const float2* Bblk = a.B + gr.b_off + (size_t)q.kb * L * G * 256;
    for (int i = q.tid; i < M; i += 256) tws[i] = a.tw[i];
    float2 xh = make_float2(0.f, 0.f), yh = make_float2(0.f, 0.f);
    if (mode != 0 && q.kvalid) {
        xh = a.Xh[(size_t)q.k * M + q.j];
        yh = a.Yh[(size_t)q.k * M + q.j];
    }
    __syncthreads();
    for (int f = q.f0; f < q.f1; ++f) {
        if (mode != 0) plane_coefs(a, gr, G, f, q.tid, coef);
        for (int base = 0; base < max(ftasks, 1); base += NTEAM) {
            const int task = base + q.team;
            const int cc = task / G, g = task - cc * G;
            const bool active = task < ftasks && q.k0 + cc < M / 2 + 1;
            float2 x[S::N1];
            load_column<M>(a, gr, G, ftasks, q.k0, f, task, q.t, x);
            if (active) fft_pass1_regs<M, -1>(q.t, xch, tws, x);
            __syncthreads();
            if (active) {
                float2* d = D + (cc * G + g) * M;
                fft_pass2<M, -1>(q.t, xch, [&](int jj, float2 v) { d[jj] = v; });
            }
            __syncthreads();
        }
        if (q.kvalid) {
            for (int l = 0; l < L; ++l) {
                float2 acc = make_float2(0.f, 0.f);
                for (int g = 0; g < G; ++g) {
                    float2 dv;
                    if (mode == 2) dv = plane_value(coef[g], xh, yh);
                    else {
                        dv = D[(q.c * G + g) * M + q.j];
                        if (mode == 1) dv = csub(dv, plane_value(coef[g], xh, yh));
                    }
                    const float2 bv = Bblk[(size_t)(l * G + g) * 256 + q.tid];
                    acc.x += bv.x * dv.x - bv.y * dv.y;
                    acc.y += bv.x * dv.y + bv.y * dv.x;
                }
                Bsp[(q.c * L + l) * M + q.j] = acc;
            }
        }
        __syncthreads();
        inverse_columns<M>(a, q, gi, L, f, tws, xch, Bsp);
    }
}

size_t cols_lds_bytes(int M, int gmax, int L) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    return ((size_t)M + (size_t)(256 / T) * N1 * (N2 + 1) + (size_t)(256 / M) * (gmax + L) * M + kMaxG) *
           sizeof(float2);
}

namespace {

template <class K>
hipError_t launch_cols_kernel(K kernel, int M, const ColArgs& a, int frames, hipStream_t s) {
    const int CPW = 256 / M, Kh = M / 2 + 1;
    const size_t lds = cols_lds_bytes(M, a.gmax, a.L);
    const dim3 grid((Kh + CPW - 1) / CPW, a.groups.count, (frames + a.frames_per_block - 1) / a.frames_per_block);
    allow_large_lds(reinterpret_cast<const void*>(kernel));
    hipLaunchKernelGGL(kernel, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

// shapes with a compile-time kernel: (M, L, laser-or-only group size, natural group size or 0)
#define SAFR_FIXED_SHAPES(X) \
    X(256, 9, 6, 3)          \
    X(256, 9, 6, 0)          \
    X(128, 5, 6, 0)          \
    X(64, 2, 4, 0)           \
    X(64, 3, 4, 0)

bool fixed_shape_known(int M, int L, int G0, int G1) {
#define SAFR_MATCH(m, l, g0, g1) \
    if (M == m && L == l && G0 == g0 && G1 == g1) return true;
    SAFR_FIXED_SHAPES(SAFR_MATCH)
#undef SAFR_MATCH
    return false;
}

}  // namespace

hipError_t launch_cols(int M, const ColArgs& a, int frames, hipStream_t s) {
    const int G0 = a.groups.g[0].G, G1 = a.groups.count > 1 ? a.groups.g[1].G : 0;
    if (a.prefetch && fixed_shape_known(M, a.L, G0, G1)) {
#define SAFR_LAUNCH(m, l, g0, g1)                           \
    if (M == m && a.L == l && G0 == g0 && G1 == g1)         \
        return launch_cols_kernel(&cols_fixed<m, l, g0, g1>, M, a, frames, s);
        SAFR_FIXED_SHAPES(SAFR_LAUNCH)
#undef SAFR_LAUNCH
    }
    switch (M) {
        case 32: return launch_cols_kernel(&cols_generic<32>, M, a, frames, s);
        case 64: return launch_cols_kernel(&cols_generic<64>, M, a, frames, s);
        case 128: return launch_cols_kernel(&cols_generic<128>, M, a, frames, s);
        case 256: return launch_cols_kernel(&cols_generic<256>, M, a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace safr
