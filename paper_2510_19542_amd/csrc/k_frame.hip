// The whole hard-real-time step (Alg. 1) of one frame in one block, for the small
// configured geometry (M = 64, n = 33, one group of 4 stars, no split tomography,
// L = 2 or 3 layers): every intermediate spectrum of a frame fits in one CU's LDS,
// so nothing but the wavefronts, B and the layers crosses the memory system (the
// three-pass path moves the row spectra R and the layer spectra C through it, about
// three times the frame's own bytes at this size).
//
// Phases of a block (512 threads = 64 teams of 8 threads, the 64-point four-step
// transforms of the other passes), separated by workgroup barriers, all in one LDS
// array U of 4 x 32 column slots of 72 float2 (72 KB, two blocks per CU):
//   1. row transforms of the pupil rows, two real rows packed per complex FFT and
//      separated into half spectra k < M/2 (the Nyquist column carries B = 0):
//      RS[g][k][row] at the start of U, the teams' exchange regions behind it;
//   2. column transforms of every star's half-spectrum column into its slot (the slot
//      is the transform's exchange buffer, then its spectrum): D[g][k][j];
//   3. apply b_l = sum_g B[l][g] d_g per frequency, in place (layer l in star slot l);
//   4. inverse column transforms of the layer columns, in place: C[l][k][p];
//   5. C2R row transforms (two rows packed per complex FFT), exchanged and staged in the
//      slots behind the layers and written out as float4 rows (in the closed loop through
//      the integrator, prev read at the pixel just before it is written).
// The arithmetic of each step is that of the three-pass path (the same transform
// routines, separation, apply and packing formulas, in the same order), so both
// give the same layers.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

namespace {

constexpr int kFM = 64, kFT = 8, kFN1 = 8, kFN2 = 8;         // transform size and its four-step shape
constexpr int kFTeams = 64, kFThreads = kFTeams * kFT;        // teams per block
constexpr int kFTL = kFN1 * (kFN2 + 1);                       // float2 per slot: a padded exchange, 16-byte multiple
constexpr int kFG = 4, kFN = 33, kFKC = kFM / 2;              // stars, pupil size, columns k < M/2
constexpr int kFP0 = (kFM - kFN + 1) / 2;                     // first pupil row and column on the grid
constexpr int kFPairs = (kFN + 1) / 2;                        // row pairs of the pupil
// pass-1 inputs of team thread t are grid indices 8 n1 + t: only n1 in [kFLO, kFHI] can meet the pupil
constexpr int kFLO = (kFP0 - kFT + 1 + kFN2 - 1) / kFN2, kFHI = (kFP0 + kFN - 1) / kFN2;
static_assert(kFM == FftShape<kFM>::N1 * FftShape<kFM>::N2 && FftShape<kFM>::T == kFT, "four-step shape");

// acc + b d as four FMAs in the order of the column pass's apply
__device__ __forceinline__ float2 fcmac(float2 acc, float2 b, float2 d) {
    acc.x = fmaf(b.x, d.x, acc.x);
    acc.x = fmaf(-b.y, d.y, acc.x);
    acc.y = fmaf(b.x, d.y, acc.y);
    acc.y = fmaf(b.y, d.x, acc.y);
    return acc;
}

}  // namespace

size_t frame_lds_bytes() { return (size_t)kFG * kFKC * kFTL * sizeof(float2); }
static_assert(kFG * kFKC * kFN + kFTeams * kFTL <= kFG * kFKC * kFTL, "row spectra and exchange regions fit U");

template <int L>
__global__ __launch_bounds__(kFThreads) void frame_kernel(FrameArgs a) {
    static_assert(L >= 1 && L <= kFG, "layers are written in place over the star slots");
    extern __shared__ float2 smem[];
    const int f = blockIdx.x;
    if (f >= a.frames) return;
    const int tid = threadIdx.x, team = tid / kFT, t = tid % kFT;
    float2* U = smem;                                 // RS [g][k][33], then slots [g][k][72], layers in place
    float2* xch = U + kFG * kFKC * kFN + team * kFTL; // row transforms: this team's exchange region
    float2 twr[kFN1];
    load_pass1_twiddles<kFM>(a.tw, t, twr);

    // 1. row transforms: task (g, pair m), rows 2m and 2m + 1 of star g
    const float* wf = a.wf + (size_t)f * kFG * kFN * kFN;
    for (int task = team; task < kFG * kFPairs; task += kFTeams) {   // whole teams: a team-uniform loop
        const int g = task / kFPairs, m = task % kFPairs;
        const int ra = 2 * m, rb = min(2 * m + 1, kFN - 1);
        const bool has_b = 2 * m + 1 < kFN;
        float2 x[kFN1];
#pragma unroll
        for (int n1 = 0; n1 < kFN1; ++n1) {
            x[n1] = make_float2(0.f, 0.f);
            if (n1 < kFLO || n1 > kFHI) continue;
            const int c = kFN2 * n1 + t - kFP0;
            const bool in = c >= 0 && c < kFN;
            const int cs = min(max(c, 0), kFN - 1);
            const float va = wf[((size_t)g * kFN + ra) * kFN + cs], vb = wf[((size_t)g * kFN + rb) * kFN + cs];
            const unsigned char ma = a.pupil[ra * kFN + cs], mb = a.pupil[rb * kFN + cs];
            x[n1] = make_float2(in && ma ? va : 0.f, in && has_b && mb ? vb : 0.f);
        }
        fft_pass1_regs<kFM, -1>(t, xch, twr, x);
        team_sync();
        float2 z[1][kFN2];
        fft_pass2_load<kFM>(t, xch, z);
        team_sync();
        fft_pass2_regs<kFM, -1>(t, z, [&](int k, float2 v) { xch[k] = v; });
        team_sync();
        // separation: A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i, for k < M/2
#pragma unroll
        for (int i = 0; i < kFKC / kFT; ++i) {
            const int k = t + kFT * i;
            const float2 zk = xch[k];
            const float2 zm = cconj(xch[(kFM - k) & (kFM - 1)]);
            float2* dst = U + ((size_t)g * kFKC + k) * kFN + ra;
            dst[0] = cscale(cadd(zk, zm), 0.5f);
            if (has_b) {
                const float2 d = csub(zk, zm);
                dst[1] = make_float2(0.5f * d.y, -0.5f * d.x);
            }
        }
        team_sync();                                  // the region is the next task's exchange buffer
    }
    __syncthreads();

    // 2. column transforms: task (g, k); every round's inputs are read before D overwrites RS
    constexpr int CR = kFG * kFKC / kFTeams;          // rounds (2)
    static_assert(CR * kFTeams == kFG * kFKC, "column tasks fill whole rounds");
    float2 xc[CR][kFN1];
#pragma unroll
    for (int r = 0; r < CR; ++r) {
        const int task = r * kFTeams + team, g = task / kFKC, k = task % kFKC;
#pragma unroll
        for (int n1 = 0; n1 < kFN1; ++n1) {
            xc[r][n1] = make_float2(0.f, 0.f);
            if (n1 < kFLO || n1 > kFHI) continue;
            const int row = kFN2 * n1 + t - kFP0;
            const bool in = row >= 0 && row < kFN;
            const float2 v = U[((size_t)g * kFKC + k) * kFN + min(max(row, 0), kFN - 1)];
            xc[r][n1] = in ? v : make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CR; ++r) {
        const int task = r * kFTeams + team, g = task / kFKC, k = task % kFKC;
        float2* col = U + ((size_t)g * kFKC + k) * kFTL;   // exchange, then spectrum
        fft_pass1_regs<kFM, -1>(t, col, twr, xc[r]);
        team_sync();
        float2 z[1][kFN2];
        fft_pass2_load<kFM>(t, col, z);
        team_sync();
        fft_pass2_regs<kFM, -1>(t, z, [&](int j, float2 v) { col[j] = v; });
    }
    __syncthreads();

    // 3. apply per frequency (k, j): the 4 star values read first, the layers written into slots l < L
#pragma unroll
    for (int i = 0; i < kFKC * kFM / kFThreads; ++i) {
        const int idx = tid + kFThreads * i, k = idx / kFM, j = idx % kFM;
        float2 d[kFG];
#pragma unroll
        for (int g = 0; g < kFG; ++g) d[g] = U[((size_t)g * kFKC + k) * kFTL + j];
        // B in the column pass's layout: [k / 4][l][g][k % 4][j]
        const float2* Bk = a.B + (size_t)(k >> 2) * L * kFG * 256 + (k & 3) * kFM + j;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int g = 0; g < kFG; ++g) acc = fcmac(acc, Bk[(l * kFG + g) * 256], d[g]);
            U[((size_t)l * kFKC + k) * kFTL + j] = acc;
        }
    }
    __syncthreads();

    // 4. inverse column transforms of the layer columns, in place
    for (int task = team; task < L * kFKC; task += kFTeams) {
        float2* col = U + (size_t)task * kFTL;        // task = l * 32 + k; the slot is the exchange buffer
        float2 x[kFN1];
#pragma unroll
        for (int n1 = 0; n1 < kFN1; ++n1) x[n1] = col[kFN2 * n1 + t];
        team_sync();
        fft_pass1_regs<kFM, +1>(t, col, twr, x);
        team_sync();
        float2 z[1][kFN2];
        fft_pass2_load<kFM>(t, col, z);
        team_sync();
        fft_pass2_regs<kFM, +1>(t, z, [&](int p, float2 v) { col[p] = v; });
    }
    __syncthreads();

    // 5. C2R rows: task (l, pair q), rows 2q and 2q + 1 packed as Z = A + i B over their Hermitian extensions;
    // the teams' exchange regions are the slots behind the layers' (as many teams as there are such slots)
    constexpr int T5 = (kFG - L) * kFKC < kFTeams ? (kFG - L) * kFKC : kFTeams;
    float2* xch5 = U + ((size_t)L * kFKC + team) * kFTL;
    for (int task = team; team < T5 && task < L * (kFM / 2); task += T5) {
        const int l = task / (kFM / 2), q = task % (kFM / 2);
        const float2* Cl = U + (size_t)l * kFKC * kFTL;     // [k][p] in slots of 72
        float2 x[kFN1];
#pragma unroll
        for (int n1 = 0; n1 < kFN1; ++n1) {
            const int kk = kFN2 * n1 + t;
            float2 z;
            if (kk == kFM / 2) {
                z = make_float2(0.f, 0.f);                    // Nyquist column: B = 0 there
            } else if (kk == 0) {
                z = make_float2(Cl[2 * q].x, Cl[2 * q + 1].x);
            } else if (kk < kFM / 2) {
                const float2 u = Cl[(size_t)kk * kFTL + 2 * q], w = Cl[(size_t)kk * kFTL + 2 * q + 1];
                z = make_float2(u.x - w.y, u.y + w.x);
            } else {
                const float2 u = Cl[(size_t)(kFM - kk) * kFTL + 2 * q], w = Cl[(size_t)(kFM - kk) * kFTL + 2 * q + 1];
                z = make_float2(u.x + w.y, w.x - u.y);
            }
            x[n1] = z;
        }
        fft_pass1_regs<kFM, +1>(t, xch5, twr, x);
        team_sync();
        float2 z[1][kFN2];
        fft_pass2_load<kFM>(t, xch5, z);
        team_sync();
        float* rows = reinterpret_cast<float*>(xch5);       // [2][M]
        fft_pass2_regs<kFM, +1>(t, z, [&](int p, float2 v) {
            rows[p] = v.x;
            rows[kFM + p] = v.y;
        });
        team_sync();
        // the two rows as float4: 32 per team, 4 per thread
#pragma unroll
        for (int i = 0; i < 2 * kFM / 4 / kFT; ++i) {
            const int e = t + kFT * i, r = e / (kFM / 4), c4 = e % (kFM / 4);
            float4 v = reinterpret_cast<const float4*>(rows)[e];
            const size_t o4 = (((size_t)f * L + l) * kFM + 2 * q + r) * (kFM / 4) + c4;
            if (a.prev) {                             // integrator of the closed loop (Alg. 3), as the output pass
                const float4 pr = reinterpret_cast<const float4*>(a.prev)[o4];
                const float keep = 1.f - a.gain;
                v.x = fmaf(a.gain, v.x, keep * pr.x);
                v.y = fmaf(a.gain, v.y, keep * pr.y);
                v.z = fmaf(a.gain, v.z, keep * pr.z);
                v.w = fmaf(a.gain, v.w, keep * pr.w);
            }
            reinterpret_cast<float4*>(a.out)[o4] = v;
        }
        team_sync();                                  // the region is the next task's exchange buffer
    }
}

bool frame_shape(int M, int n, int G, int L, int mode) {
    return M == kFM && n == kFN && G == kFG && mode == 0 && (L == 2 || L == 3);
}

hipError_t launch_frame(const FrameArgs& a, int L, hipStream_t s) {
    const size_t lds = frame_lds_bytes();
    const void* k = L == 2 ? reinterpret_cast<const void*>(&frame_kernel<2>)
                           : reinterpret_cast<const void*>(&frame_kernel<3>);
    allow_large_lds(k);
    if (L == 2) hipLaunchKernelGGL(frame_kernel<2>, dim3(a.frames), dim3(kFThreads), lds, s, a);
    else if (L == 3) hipLaunchKernelGGL(frame_kernel<3>, dim3(a.frames), dim3(kFThreads), lds, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace safr
