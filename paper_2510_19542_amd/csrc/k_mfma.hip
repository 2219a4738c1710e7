// Batched column pass with the per-frequency apply on BF16 matrix cores.
//
// For one frequency n the apply b = B_n d (L x G complex) is the real-split
// product [Re b; Im b] = [[Re B, -Im B], [Im B, Re B]] [Re d; Im d] of a
// 2L x 2G real matrix with 2G real values per frame.  With the frames as the
// N dimension it becomes a GEMM per frequency; P frequencies are packed
// block-diagonally into one 16 x 32 A tile of v_mfma_f32_16x16x32_bf16
// (rows: P frequencies x 2Lt layer rows; columns: P frequencies x 2G star
// values; Lt <= 8 layers per tile), and the 16 columns of the B operand are 16
// frames.  Precision: both operands are split into bf16 hi + lo (x_lo = bf16(x -
// x_hi)); three products hi*hi + hi*lo + lo*hi are accumulated in FP32 (the
// lo*lo term, ~2^-16 relative, is dropped).  The A tiles (hi and lo) are built
// once per plan from the FP32 B by pack_kernel, already in the lane layout of
// the instruction: lane l holds A[l % 16][8 (l / 16) + v], v = 0..7.
//
// The column FFTs before and after the apply and the tip/tilt handling are the
// same as in the FP32 column pass; one block owns one column and NF frames.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

}  // namespace

// A tiles: per group [k][q][t][hi, lo][lane 64][8] bf16 (q: frequency group of P, t: layer tile)
__global__ void pack_kernel(int M, int L, int G, int lt, int ntile, int ppm, const float2* __restrict__ B32,
                            __bf16* __restrict__ Apack) {
    const int Kh = M / 2 + 1, cpw = 256 / M, nq = M / ppm;
    const size_t tiles = (size_t)Kh * nq * ntile;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;      // one (tile, lane) per thread
    if (e >= tiles * 64) return;
    const int lane = (int)(e % 64);
    const size_t tile = e / 64;
    const int t = (int)(tile % ntile);
    const int q = (int)((tile / ntile) % nq);
    const int k = (int)(tile / ((size_t)ntile * nq));
    const int i = lane % 16;
    const int p = i / (2 * lt), r = i % (2 * lt);
    const int l = t * lt + (r % lt);
    __bf16 hi[8], lo[8];
    for (int v = 0; v < 8; ++v) {
        const int kk = 8 * (lane / 16) + v;
        const int p2 = kk / (2 * G), s = kk % (2 * G);
        float val = 0.f;
        if (p < ppm && p == p2 && l < L && i < ppm * 2 * lt && kk < ppm * 2 * G) {
            const int g = s % G, j = q * ppm + p;
            const float2 b = B32[((((size_t)(k / cpw) * L + l) * G + g) * cpw + (k % cpw)) * M + j];
            const bool re_row = r < lt, re_col = s < G;
            val = re_row ? (re_col ? b.x : -b.y) : (re_col ? b.y : b.x);
        }
        split_bf16(val, hi[v], lo[v]);
    }
    __bf16* o = Apack + ((tile * 2) * 64 + lane) * 8;
    for (int v = 0; v < 8; ++v) {
        o[v] = hi[v];
        o[64 * 8 + v] = lo[v];
    }
}

hipError_t launch_pack_bf16(int M, int L, int G, const float2* B32, uint16_t* Apack, int lt, int ntile, int ppm,
                            hipStream_t s) {
    const size_t tiles = (size_t)(M / 2 + 1) * (M / ppm) * ntile;
    const size_t threads = tiles * 64;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, M, L, G, lt, ntile, ppm,
                       B32, reinterpret_cast<__bf16*>(Apack));
    return hipGetLastError();
}

template <int M, int NF>
__global__ __launch_bounds__(256) void cols_mfma_kernel(MfmaArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T, Kh = M / 2 + 1, NTEAM = 256 / T, TL = team_lds<M>();
    extern __shared__ float2 smem[];
    const int k = blockIdx.x;
    const int fb = blockIdx.z * NF;
    const int nf = min(NF, a.frames - fb);
    const GroupArgs& gr = a.grp;
    const int G = gr.G, mode = gr.mode, L = a.L, n = a.n;
    const int lt = a.lt, ntile = a.ntile, ppm = a.ppm;
    const int tid = threadIdx.x, team = tid / T, t = tid % T;
    const int lane = tid & 63, wave = tid >> 6;

    float2* tws = smem;                                    // [M]
    float2* xch = tws + M + team * TL;                     // [NTEAM][TL]
    float2* D = tws + M + NTEAM * TL;                      // [NF][G][M]
    float2* Bsp = D + NF * G * M;                          // [NF][L][M]
    float2* coef = Bsp + NF * L * M;                       // [NF][G]

    for (int i = tid; i < M; i += 256) tws[i] = a.tw[i];
    if (mode != 0) {
        const PlaneArgs pa{a.planes, a.plane_nch, a.J, G, fb, fb + nf, nf * G, 0};   // nf = valid frames of the block
        float2 pl[1];
        plane_fetch<1>(pa, pl);
        plane_put<1>(pa, pl, coef);
    }
    __syncthreads();

    // 1. forward column transforms of the NF frames
    const int ftasks = nf * G;
    for (int base = 0; base < ftasks; base += NTEAM) {
        const int task = base + team;
        const bool active = task < ftasks;
        const int f = task / G, g = task % G;
        if (active) {
            const float2* col = a.R + (((size_t)(fb + f) * a.J + g) * Kh + k) * n;   // group slot g
            fft_pass1<M, -1>(t, xch, tws, [&](int p) -> float2 {
                const int pr = p - a.p0;
                return (pr >= 0 && pr < n) ? col[pr] : make_float2(0.f, 0.f);
            });
        }
        __syncthreads();
        if (active) {
            float2* d = D + (f * G + g) * M;
            fft_pass2<M, -1>(t, xch, [&](int j, float2 v) { d[j] = v; });
        }
        __syncthreads();
    }

    // 2. apply on matrix cores: one wave per (layer tile, frequency group) item
    const bf16x8_t* Ap = reinterpret_cast<const bf16x8_t*>(a.Apack);
    const int nq = M / ppm;
    const int fl = lane % 16;                          // frame of this lane's B-operand column and D column
    float* bspf = reinterpret_cast<float*>(Bsp);
    for (int item = wave; item < ntile * nq; item += 4) {
        const int tt = item / nq, q = item % nq;
        const size_t tile = ((size_t)k * nq + q) * ntile + tt;
        const bf16x8_t ahi = Ap[(tile * 2) * 64 + lane];
        const bf16x8_t alo = Ap[(tile * 2 + 1) * 64 + lane];
        bf16x8_t xhi, xlo;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int kk = 8 * (lane / 16) + v;
            const int p = kk / (2 * G), s = kk % (2 * G);
            float val = 0.f;
            if (fl < nf && p < ppm) {
                const int g = s % G, j = q * ppm + p;
                float2 d = D[(fl * G + g) * M + j];
                if (mode != 0) {
                    const float2 cf = coef[fl * G + g];
                    const float2 xh = a.Xh[(size_t)k * M + j], yh = a.Yh[(size_t)k * M + j];
                    d = csub(d, make_float2(cf.x * xh.x + cf.y * yh.x, cf.x * xh.y + cf.y * yh.y));
                }
                val = s < G ? d.x : d.y;
            }
            __bf16 h, lo;
            split_bf16(val, h, lo);
            xhi[v] = h;
            xlo[v] = lo;
        }
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, xhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, xlo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, xhi, acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * (lane / 16) + v;
            const int p = i / (2 * lt), r = i % (2 * lt);
            const int l = tt * lt + (r % lt);
            if (fl < nf && p < ppm && l < L) {
                const int j = q * ppm + p;
                bspf[2 * ((fl * L + l) * M + j) + (r < lt ? 0 : 1)] = acc[v];
            }
        }
    }
    __syncthreads();

    // 3. inverse column transforms
    const int itasks = nf * L;
    for (int base = 0; base < itasks; base += NTEAM) {
        const int task = base + team;
        const bool active = task < itasks;
        const int f = task / L, l = task % L;
        if (active) {
            const float2* src = Bsp + (f * L + l) * M;
            fft_pass1<M, +1>(t, xch, tws, [&](int j) -> float2 { return src[j]; });
        }
        __syncthreads();
        if (active) {
            float2* dst = a.C + c_index(fb + f, l, L, M, k, 0);
            fft_pass2<M, +1>(t, xch, [&](int p, float2 v) { dst[(size_t)(p >> 3) * (Kh * 8) + (p & 7)] = v; });
        }
        __syncthreads();
    }
}

size_t mfma_lds_bytes(int M, int NF, int G, int L) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    return ((size_t)M + (size_t)(256 / T) * N1 * (N2 + 1) + (size_t)NF * G * M + (size_t)NF * L * M +
            (size_t)NF * G) * sizeof(float2);
}

namespace {

template <int M, int NF>
hipError_t launch_mfma_t(const MfmaArgs& a, int frames, hipStream_t s) {
    const size_t lds = mfma_lds_bytes(M, NF, a.grp.G, a.L);
    allow_large_lds(reinterpret_cast<const void*>(&cols_mfma_kernel<M, NF>));
    const dim3 grid(M / 2, 1, (frames + NF - 1) / NF);     // the Nyquist column (B = 0) is left out
    hipLaunchKernelGGL((cols_mfma_kernel<M, NF>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int M>
hipError_t launch_mfma_m(const MfmaArgs& a, int frames, int nf, hipStream_t s) {
    switch (nf) {
        case 16: return launch_mfma_t<M, 16>(a, frames, s);
        case 8: return launch_mfma_t<M, 8>(a, frames, s);
        case 4: return launch_mfma_t<M, 4>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_cols_mfma(int M, const MfmaArgs& a, int frames, int frames_per_block, hipStream_t s) {
    switch (M) {
        case 32: return launch_mfma_m<32>(a, frames, frames_per_block, s);
        case 64: return launch_mfma_m<64>(a, frames, frames_per_block, s);
        case 128: return launch_mfma_m<128>(a, frames, frames_per_block, s);
        default: return hipErrorNotSupported;
    }
}

}  // namespace safr
