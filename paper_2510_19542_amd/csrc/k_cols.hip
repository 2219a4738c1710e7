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
// B slice is one contiguous run and thread t owns the entries t, t + 256, ...:
// they are loaded into registers once, at entry (overlapping the first column
// FFT), and reused for every frame of the chunk.
//
// Split tomography (Sec. 3.3): the least-squares plane b x + c y of each
// wavefront over the pupil is obtained from the moments written by the row
// pass; since the transform is linear, removing the plane (laser stars) is
// d_g -= b DFT2(x mask) + c DFT2(y mask) and keeping only the plane (natural
// stars) is d_g = b DFT2(x mask) + c DFT2(y mask), with the two transforms
// precomputed in FP64 per plan.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

template <int M, int GLMAX>
__global__ __launch_bounds__(256) void cols_kernel(ColArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T;
    constexpr int CPW = 256 / M;
    constexpr int Kh = M / 2 + 1;
    constexpr int NTEAM = 256 / T;
    constexpr int TL = team_lds<M>();
    extern __shared__ float2 smem[];

    const int gi = blockIdx.y;
    const int kb = blockIdx.x;
    const int k0 = kb * CPW;
    const GroupArgs& gr = a.groups.g[gi];
    const int G = gr.G;
    const int mode = gr.mode;
    const int L = a.L;
    const int LG = L * G;
    const int n = a.n;
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid % T;
    const int c = tid / M, j = tid % M;
    const int k = k0 + c;
    const bool kvalid = k < Kh;
    const int f0 = blockIdx.z * a.frames_per_block;
    const int f1 = min(a.frames, f0 + a.frames_per_block);

    float2* xch = smem + team * TL;
    float2* D = smem + NTEAM * TL;               // [CPW][G][M]
    float2* Bsp = D + CPW * a.gmax * M;          // [CPW][L][M]
    float2* coef = Bsp + CPW * L * M;            // [G] plane coefficients (b, c)

    const float2* Bblk = a.B + gr.b_off + (size_t)kb * LG * 256;
    const int ftasks = mode == 2 ? 0 : CPW * G;       // natural stars of a mixed asterism need no transform

    // inputs of one pass-1 sub-transform of the column FFT: x[n1] = column[N2 n1 + t]
    float2 x[S::N1];
    auto load_column = [&](int f, int task) {
        const int cc = task / G, g = task - cc * G;
        const int kk = k0 + cc;
        if (task < ftasks && kk < Kh) {
            const float2* col = a.R + (((size_t)f * a.J + gr.star[g]) * Kh + kk) * n;
#pragma unroll
            for (int n1 = 0; n1 < S::N1; ++n1) {
                const int pr = S::N2 * n1 + t - a.p0;
                x[n1] = (pr >= 0 && pr < n) ? col[pr] : make_float2(0.f, 0.f);
            }
        }
    };
    // the first transform's inputs are requested before B: loads retire in order, so the
    // first column FFT does not wait for the B slice, which stays in registers for every frame
    load_column(f0, team);
    float2 breg[GLMAX > 0 ? GLMAX : 1];
    if constexpr (GLMAX > 0) {
#pragma unroll
        for (int i = 0; i < GLMAX; ++i)
            breg[i] = (i < LG) ? Bblk[(size_t)i * 256 + tid] : make_float2(0.f, 0.f);
    }
    float2 xh = make_float2(0.f, 0.f), yh = make_float2(0.f, 0.f);
    if (mode != 0 && kvalid) {
        xh = a.Xh[(size_t)k * M + j];
        yh = a.Yh[(size_t)k * M + j];
    }

    for (int f = f0; f < f1; ++f) {
        if (mode != 0 && tid < G) {
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
        // 1. forward column transforms
        for (int base = 0; base < max(ftasks, 1); base += NTEAM) {
            const int task = base + team;
            const int cc = task / G, g = task - cc * G;
            const bool active = task < ftasks && k0 + cc < Kh;
            if (f != f0 || base != 0) load_column(f, task);
            if (active) fft_pass1_regs<M, -1>(t, xch, a.tw, x);
            __syncthreads();
            if (active) {
                float2* d = D + (cc * G + g) * M;
                fft_pass2<M, -1>(t, xch, [&](int jj, float2 v) { d[jj] = v; });
            }
            __syncthreads();
        }

        // 2. per-frequency apply
        if (kvalid) {
            const float2* d = D + c * G * M + j;
            float2* bo = Bsp + c * L * M + j;
            auto dval = [&](int g) -> float2 {
                if (mode == 0) return d[g * M];
                const float2 cf = coef[g];
                const float2 plane = make_float2(cf.x * xh.x + cf.y * yh.x, cf.x * xh.y + cf.y * yh.y);
                return mode == 2 ? plane : csub(d[g * M], plane);
            };
            if constexpr (GLMAX > 0) {
                float2 acc = make_float2(0.f, 0.f);
                int g = 0, l = 0;
#pragma unroll
                for (int i = 0; i < GLMAX; ++i) {
                    if (i < LG) {
                        const float2 bv = breg[i];
                        const float2 dv = dval(g);
                        acc.x += bv.x * dv.x - bv.y * dv.y;
                        acc.y += bv.x * dv.y + bv.y * dv.x;
                        if (++g == G) {
                            bo[l * M] = acc;
                            acc = make_float2(0.f, 0.f);
                            g = 0;
                            ++l;
                        }
                    }
                }
            } else {
                for (int l = 0; l < L; ++l) {
                    float2 acc = make_float2(0.f, 0.f);
                    for (int g = 0; g < G; ++g) {
                        const float2 bv = Bblk[(size_t)(l * G + g) * 256 + tid];
                        const float2 dv = dval(g);
                        acc.x += bv.x * dv.x - bv.y * dv.y;
                        acc.y += bv.x * dv.y + bv.y * dv.x;
                    }
                    bo[l * M] = acc;
                }
            }
        }
        __syncthreads();

        // 3. inverse column transforms
        const int itasks = CPW * L;
        for (int base = 0; base < itasks; base += NTEAM) {
            const int task = base + team;
            const int cc = task / L, l = task - cc * L;
            const int kk = k0 + cc;
            const bool active = task < itasks && kk < Kh;
            if (active) {
                const float2* src = Bsp + (cc * L + l) * M;
                fft_pass1<M, +1>(t, xch, a.tw, [&](int jj) -> float2 { return src[jj]; });
            }
            __syncthreads();
            if (active) {
                float2* dst = a.C + ((((size_t)f * a.groups.count + gi) * L + l) * Kh + kk) * M;
                fft_pass2<M, +1>(t, xch, [&](int p, float2 v) { dst[p] = v; });
            }
            __syncthreads();
        }
    }
}

template <int M, int GLMAX>
static hipError_t launch_cols_t2(const ColArgs& a, int frames, hipStream_t s) {
    constexpr int CPW = 256 / M;
    constexpr int Kh = M / 2 + 1;
    const size_t lds = ((size_t)(256 / FftShape<M>::T) * team_lds<M>() + (size_t)CPW * (a.gmax + a.L) * M +
                        kMaxG) * sizeof(float2);
    const dim3 grid((Kh + CPW - 1) / CPW, a.groups.count, (frames + a.frames_per_block - 1) / a.frames_per_block);
    allow_large_lds(reinterpret_cast<const void*>(&cols_kernel<M, GLMAX>));
    hipLaunchKernelGGL((cols_kernel<M, GLMAX>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int M>
static hipError_t launch_cols_t(const ColArgs& a, int frames, hipStream_t s) {
    int lg = 0;
    for (int i = 0; i < a.groups.count; ++i) lg = lg > a.L * a.groups.g[i].G ? lg : a.L * a.groups.g[i].G;
    if (!a.prefetch) return launch_cols_t2<M, 0>(a, frames, s);
    if (lg <= 8) return launch_cols_t2<M, 8>(a, frames, s);
    if (lg <= 16) return launch_cols_t2<M, 16>(a, frames, s);
    if (lg <= 32) return launch_cols_t2<M, 32>(a, frames, s);
    if (lg <= 48) return launch_cols_t2<M, 48>(a, frames, s);
    if (lg <= 56) return launch_cols_t2<M, 56>(a, frames, s);
    if (lg <= 64) return launch_cols_t2<M, 64>(a, frames, s);
    return launch_cols_t2<M, 0>(a, frames, s);
}

hipError_t launch_cols(int M, const ColArgs& a, int frames, hipStream_t s) {
    switch (M) {
        case 32: return launch_cols_t<32>(a, frames, s);
        case 64: return launch_cols_t<64>(a, frames, s);
        case 128: return launch_cols_t<128>(a, frames, s);
        case 256: return launch_cols_t<256>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

size_t cols_lds_bytes(int M, int gmax, int L) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    return ((size_t)(256 / T) * N1 * (N2 + 1) + (size_t)(256 / M) * (gmax + L) * M + kMaxG) * sizeof(float2);
}

}  // namespace safr
