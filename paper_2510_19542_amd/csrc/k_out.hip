// Output pass of SAFR's hard-real-time step (Alg. 1, last loop), fused with the
// split-tomography sum (Sec. 3.3):
//   - C2R row transforms of the layer spectra C[f][grp][l][k][p] (two real rows
//     packed into one complex inverse FFT), scaled by 1/M^2 (IDFT2 of Sec. 3.2);
//   - mixed asterisms: the natural-star layer (grid spacing pitch) is resampled
//     bilinearly and periodically at the laser layer grid points (spacing
//     c_l * pitch), i.e. at fractional index u = c_l (p - M/2) + M/2, and added.
// One block of 256 threads writes RT output rows of one layer of one frame; the
// natural-star rows it needs (at most RT + 1, since c_l <= 1) are transformed
// in the same block.  All global loads of a phase are issued before any is used.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

template <int M, int RT, bool MIXED>
__global__ __launch_bounds__(256) void out_kernel(OutArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T;
    constexpr int Kh = M / 2 + 1;
    constexpr int NTEAM = 256 / T;
    constexpr int TL = team_lds<M>();
    constexpr int NS = MIXED ? RT + 2 : 0;             // natural-star row slots
    constexpr int TR = RT + NS;
    extern __shared__ float2 smem[];

    const int l = blockIdx.y;
    const int f = blockIdx.z;
    const int r0 = blockIdx.x * RT;
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid % T;
    const float cl = a.c[l];
    const float hm = 0.5f * (float)M;

    float2* tws = smem;                                         // [M]
    float2* xch = tws + M + team * TL;                          // [NTEAM][TL]
    float2* tile = tws + M + NTEAM * TL;                        // [TR][Kh]
    float* real = reinterpret_cast<float*>(tile + TR * Kh);     // [TR][M]

    int nlo = 0, nrows = 0;
    if (MIXED) {
        nlo = (int)floorf(cl * ((float)r0 - hm) + hm);
        const int nhi = (int)floorf(cl * ((float)(r0 + RT - 1) - hm) + hm) + 1;
        nrows = nhi - nlo + 1;                                  // <= RT + 1
    }

    const size_t lstride = (size_t)Kh * M;
    const float2* Cl = a.C + ((size_t)f * a.groups + 0) * a.L * lstride + (size_t)l * lstride;
    const float2* Cn = a.C + ((size_t)f * a.groups + a.ngs_group) * a.L * lstride + (size_t)l * lstride;

    // issue every load of the block, then store to LDS: twiddles, laser rows, natural rows
    constexpr int NL = (Kh * RT + 255) / 256;
    constexpr int NN = (Kh * NS + 255) / 256;
    const float2 twv = tid < M ? a.tw[tid] : make_float2(0.f, 0.f);
    float2 vl[NL], vn[NN > 0 ? NN : 1];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int idx = tid + 256 * i;                          // r fastest: RT consecutive values per k
        if (idx < Kh * RT) vl[i] = Cl[(size_t)(idx / RT) * M + r0 + (idx % RT)];
    }
    if constexpr (MIXED) {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx / NS, r = idx % NS;
            if (idx < Kh * NS && r < nrows) vn[i] = Cn[(size_t)k * M + ((nlo + r) & (M - 1))];
        }
    }
    if (tid < M) tws[tid] = twv;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int idx = tid + 256 * i;
        if (idx < Kh * RT) tile[(idx % RT) * Kh + idx / RT] = vl[i];
    }
    if constexpr (MIXED) {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx / NS, r = idx % NS;
            if (idx < Kh * NS && r < nrows) tile[(RT + r) * Kh + k] = vn[i];
        }
    }
    __syncthreads();

    // packed C2R: Z[q] = A[q] + i B[q] over the Hermitian extension of the two rows
    const float scale = 1.0f / ((float)M * (float)M);
    constexpr int LP = RT / 2;
    const int np = (nrows + 1) / 2;
    const int tasks = LP + np;
    for (int base = 0; base < tasks; base += NTEAM) {
        const int task = base + team;
        const bool active = task < tasks;
        int ra = 0, rb = -1;
        if (active) {
            if (task < LP) {
                ra = 2 * task;
                rb = ra + 1;
            } else {
                ra = RT + 2 * (task - LP);
                rb = (2 * (task - LP) + 1 < nrows) ? ra + 1 : -1;
            }
            const float2* A = tile + ra * Kh;
            const float2* Bv = tile + (rb >= 0 ? rb : ra) * Kh;
            const bool hb = rb >= 0;
            fft_pass1<M, +1>(t, xch, tws, [&](int q) -> float2 {
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
#pragma unroll
    for (int i = 0; i < (RT * M + 255) / 256; ++i) {
        const int idx = tid + 256 * i;
        if (idx >= RT * M) break;
        const int r = idx / M, q = idx % M;
        float v = real[r * M + q];
        if constexpr (MIXED) {
            const float u = cl * ((float)(r0 + r) - hm) + hm;
            const float w = cl * ((float)q - hm) + hm;
            const float fu0 = floorf(u), fw0 = floorf(w);
            const float fu = u - fu0, fw = w - fw0;
            const int i0 = min(max((int)fu0 - nlo, 0), nrows - 2);
            const int j0 = ((int)fw0) & (M - 1);
            const int j1 = (j0 + 1) & (M - 1);
            const float* n0 = real + (size_t)(RT + i0) * M;
            const float* n1 = n0 + M;
            const float top = (1.f - fw) * n0[j0] + fw * n0[j1];
            const float bot = (1.f - fw) * n1[j0] + fw * n1[j1];
            v += (1.f - fu) * top + fu * bot;
        }
        out[(size_t)r * M + q] = v;
    }
}

size_t out_lds_bytes(int M, int RT, bool mixed) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    const int TR = RT + (mixed ? RT + 2 : 0);
    return ((size_t)M + (size_t)(256 / T) * N1 * (N2 + 1) + (size_t)TR * (M / 2 + 1)) * sizeof(float2) +
           (size_t)TR * M * sizeof(float);
}

namespace {

template <int M, int RT, bool MIXED>
hipError_t launch_out_t(const OutArgs& a, int frames, hipStream_t s) {
    const size_t lds = out_lds_bytes(M, RT, MIXED);
    allow_large_lds(reinterpret_cast<const void*>(&out_kernel<M, RT, MIXED>));
    hipLaunchKernelGGL((out_kernel<M, RT, MIXED>), dim3(M / RT, a.L, frames), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int M, bool MIXED>
hipError_t launch_out_rt(const OutArgs& a, int frames, hipStream_t s) {
    switch (a.rows_per_block) {
        case 2: return launch_out_t<M, 2, MIXED>(a, frames, s);
        case 4: return launch_out_t<M, 4, MIXED>(a, frames, s);
        case 8: return launch_out_t<M, 8, MIXED>(a, frames, s);
        case 16: return launch_out_t<M, 16, MIXED>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

template <int M>
hipError_t launch_out_m(const OutArgs& a, int frames, hipStream_t s) {
    return a.mixed ? launch_out_rt<M, true>(a, frames, s) : launch_out_rt<M, false>(a, frames, s);
}

}  // namespace

hipError_t launch_out(int M, const OutArgs& a, int frames, hipStream_t s) {
    switch (M) {
        case 32: return launch_out_m<32>(a, frames, s);
        case 64: return launch_out_m<64>(a, frames, s);
        case 128: return launch_out_m<128>(a, frames, s);
        case 256: return launch_out_m<256>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace safr
