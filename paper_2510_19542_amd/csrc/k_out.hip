// Output pass of SAFR's hard-real-time step (Alg. 1, last loop), fused with the
// split-tomography sum (Sec. 3.3):
//   - C2R row transforms of the layer spectra C[f][grp][l][k][p] (two real rows
//     packed into one complex inverse FFT), scaled by 1/M^2 (IDFT2 of Sec. 3.2);
//   - mixed asterisms: the natural-star layer (grid spacing pitch) is resampled
//     bilinearly and periodically at the laser layer grid points (spacing
//     c_l * pitch), i.e. at fractional index u = c_l (p - M/2) + M/2, and added.
// One block of 256 threads writes `rows_per_block` output rows of one layer of
// one frame; the natural-star rows it needs (at most rows_per_block + 1, since
// c_l <= 1) are transformed in the same block.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

template <int M>
__global__ __launch_bounds__(256) void out_kernel(OutArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T;
    constexpr int Kh = M / 2 + 1;
    constexpr int NTEAM = 256 / T;
    constexpr int TL = team_lds<M>();
    extern __shared__ float2 smem[];

    const int l = blockIdx.y;
    const int f = blockIdx.z;
    const int RT = a.rows_per_block;
    const int r0 = blockIdx.x * RT;
    const int rows = min(RT, M - r0);
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid % T;
    const float cl = a.c[l];
    const float hm = 0.5f * (float)M;

    // natural-star rows needed by the bilinear resample
    int nlo = 0, nrows = 0;
    if (a.mixed) {
        nlo = (int)floorf(cl * ((float)r0 - hm) + hm);
        const int nhi = (int)floorf(cl * ((float)(r0 + rows - 1) - hm) + hm) + 1;
        nrows = nhi - nlo + 1;
    }
    const int trows = rows + nrows;

    float2* xch = smem + team * TL;
    float2* tile = smem + NTEAM * TL;                        // [trows][Kh]
    float* real = reinterpret_cast<float*>(tile + (size_t)trows * Kh);   // [trows][M]

    const size_t lstride = (size_t)Kh * M;
    const float2* Cl = a.C + ((size_t)f * a.groups + 0) * a.L * lstride + (size_t)l * lstride;
    const float2* Cn = a.C + ((size_t)f * a.groups + a.ngs_group) * a.L * lstride + (size_t)l * lstride;

    // load the row slices: tile[r][k] = C[k][row r]
    for (int idx = tid; idx < Kh * rows; idx += 256) {
        const int k = idx / rows, r = idx % rows;
        tile[r * Kh + k] = Cl[(size_t)k * M + r0 + r];
    }
    for (int idx = tid; idx < Kh * nrows; idx += 256) {
        const int k = idx / nrows, r = idx % nrows;
        tile[(rows + r) * Kh + k] = Cn[(size_t)k * M + ((nlo + r) & (M - 1))];
    }
    __syncthreads();

    // packed C2R: Z[q] = A[q] + i B[q] for the Hermitian extension of the two rows
    const float scale = 1.0f / ((float)M * (float)M);
    const int lp = (rows + 1) / 2, np = (nrows + 1) / 2;
    const int tasks = lp + np;
    for (int base = 0; base < tasks; base += NTEAM) {
        const int task = base + team;
        const bool active = task < tasks;
        int ra = 0, rb = -1;
        if (active) {
            if (task < lp) {
                ra = 2 * task;
                rb = (2 * task + 1 < rows) ? ra + 1 : -1;
            } else {
                ra = rows + 2 * (task - lp);
                rb = (2 * (task - lp) + 1 < nrows) ? ra + 1 : -1;
            }
            const float2* A = tile + ra * Kh;
            const float2* Bv = tile + (rb >= 0 ? rb : ra) * Kh;
            const bool hb = rb >= 0;
            fft_pass1<M, +1>(t, xch, a.tw, [&](int q) -> float2 {
                if (q == 0 || q == M / 2) return make_float2(A[q].x, hb ? Bv[q].x : 0.f);
                if (q < M / 2) {
                    const float2 x = A[q];
                    const float2 y = hb ? Bv[q] : make_float2(0.f, 0.f);
                    return make_float2(x.x - y.y, x.y + y.x);
                }
                const float2 x = A[M - q];
                const float2 y = hb ? Bv[M - q] : make_float2(0.f, 0.f);
                return make_float2(x.x + y.y, y.x - x.y);
            });
        }
        __syncthreads();
        if (active) {
            float* oa = real + (size_t)ra * M;
            float* ob = real + (size_t)(rb >= 0 ? rb : ra) * M;
            const bool hb = rb >= 0;
            fft_pass2<M, +1>(t, xch, [&](int p, float2 v) {
                oa[p] = v.x * scale;
                if (hb) ob[p] = v.y * scale;
            });
        }
        __syncthreads();
    }

    // write rows (+ resampled natural-star layer)
    float* out = a.out + (((size_t)f * a.L + l) * M + r0) * M;
    for (int idx = tid; idx < rows * M; idx += 256) {
        const int r = idx / M, q = idx % M;
        float v = real[r * M + q];
        if (a.mixed) {
            const float u = cl * ((float)(r0 + r) - hm) + hm;
            const float w = cl * ((float)q - hm) + hm;
            const float fu0 = floorf(u), fw0 = floorf(w);
            const float fu = u - fu0, fw = w - fw0;
            const int i0 = min(max((int)fu0 - nlo, 0), nrows - 2);
            const int j0 = ((int)fw0) & (M - 1);
            const int j1 = (j0 + 1) & (M - 1);
            const float* n0 = real + (size_t)(rows + i0) * M;
            const float* n1 = n0 + M;
            const float top = (1.f - fw) * n0[j0] + fw * n0[j1];
            const float bot = (1.f - fw) * n1[j0] + fw * n1[j1];
            v += (1.f - fu) * top + fu * bot;
        }
        out[(size_t)r * M + q] = v;
    }
}

template <int M>
static hipError_t launch_out_t(const OutArgs& a, int frames, hipStream_t s) {
    constexpr int Kh = M / 2 + 1;
    const int RT = a.rows_per_block;
    const int trows = a.mixed ? 2 * RT + 2 : RT;
    const size_t lds = (size_t)(256 / FftShape<M>::T) * team_lds<M>() * sizeof(float2) +
                       (size_t)trows * Kh * sizeof(float2) + (size_t)trows * M * sizeof(float);
    const dim3 grid((M + RT - 1) / RT, a.L, frames);
    allow_large_lds(reinterpret_cast<const void*>(&out_kernel<M>));
    hipLaunchKernelGGL(out_kernel<M>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_out(int M, const OutArgs& a, int frames, hipStream_t s) {
    switch (M) {
        case 32: return launch_out_t<32>(a, frames, s);
        case 64: return launch_out_t<64>(a, frames, s);
        case 128: return launch_out_t<128>(a, frames, s);
        case 256: return launch_out_t<256>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace safr
