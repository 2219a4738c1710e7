// Row pass of the forward 2-D transform (Alg. 1, first loop).
//
// The zero-extended M x M wavefront has only n nonzero rows and columns, so
// only the n pupil rows are transformed; two real rows are packed into one
// complex M-point FFT (z = a + i b) and separated afterwards with
// A[k] = (Z[k] + conj Z[-k]) / 2,  B[k] = (Z[k] - conj Z[-k]) / (2 i).
// Output: R[f][slot][k][row] (the star's group slot) for k < M/2 (the half spectrum without its Nyquist
// column, which B ignores; R keeps a slot for it), rows contiguous so the column
// pass reads each column as one run.  Each team takes its two rows from global
// memory straight into the registers of the first transform pass.
//
// Split tomography (Sec. 3.3) needs the least-squares tip/tilt plane of each
// wavefront over the pupil.  Its coefficients are linear in the data, so each
// block forms those of its own rows from their moments (sum v, sum x v, sum y v)
// and the passes that use the plane add the chunks' parts as they read them: the
// column pass to remove the plane of the laser stars in the Fourier domain, the
// output pass to add the natural stars' layers.  Natural stars of a mixed
// asterism therefore need no row transform.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

// NN > 0: the pupil size at compile time (the configured workloads); only the inputs that can fall inside
// the pupil columns are loaded.  All loads are issued unconditionally (addresses clamped into the block's
// rows, values outside the pupil or past the chunk selected away), so the compiler can wait for them as a
// group instead of one at a time behind branches.
template <int M, int NN>
__global__ __launch_bounds__(256) void rows_kernel(RowArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T, N1 = S::N1, N2 = S::N2;
    constexpr int Kh = M / 2 + 1;
    constexpr int KC = M / 2;                       // columns written: the Nyquist column is not used
    constexpr int TS = team_lds<M>() + 2;           // team region stride, 4 banks apart
    constexpr int P0 = NN > 0 ? (M - NN + 1) / 2 : 0;
    // grid column N2 n1 + t (t < T = N2) meets the pupil columns p0 .. p0 + n - 1 only for n1 in [WLO, WHI]
    constexpr int WLO = NN > 0 && P0 - N2 + 1 > 0 ? (P0 - N2 + 1 + N2 - 1) / N2 : 0;
    constexpr int WHI = NN > 0 ? ((P0 + NN - 1) / N2 < N1 - 1 ? (P0 + NN - 1) / N2 : N1 - 1) : N1 - 1;
    static_assert(T == N2, "one pass-1 sub-transform per team thread");
    extern __shared__ float2 smem[];

    const int n = NN > 0 ? NN : a.n;
    const int p0 = NN > 0 ? P0 : a.p0;
    const int star = blockIdx.y;
    const int f = blockIdx.z;
    const int chunk = blockIdx.x;
    const int r0 = chunk * a.rows_per_block;
    const int rows = min(a.rows_per_block, n - r0);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int team = tid / T;
    const int t = tid % T;
    const int nteams = a.rows_per_block / 2;       // one row pair per team: the chunk is one round
    const int mode = a.tt_mode[star];
    const float* wf = a.wf + ((size_t)f * a.J + star) * (size_t)n * n + (size_t)r0 * n;
    const unsigned char* pup = a.pupil + (size_t)r0 * n;

    // LDS: one region per team (the pass-1 -> pass-2 exchange, then the packed spectrum), 3 floats per
    // wavefront for the moment reduction.  The thread's pass-1 twiddles are held in registers (no LDS table,
    // so more blocks fit a CU)
    float2* xch = smem + team * TS;
    float* red = reinterpret_cast<float*>(smem + nteams * TS);

    // the thread's twiddles, then the team's two pupil-masked rows straight into the pass-1 registers:
    // x[n1] = (row a, row b) at grid column N2 n1 + t, i.e. pupil column N2 n1 + t - p0 (all loads issued
    // before any is used)
    float2 twr[N1];
    load_pass1_twiddles<M>(a.tw, t, twr);
    const int ra = 2 * team;
    const bool active = team < nteams && ra < rows;
    const bool has_b = active && ra + 1 < rows;
    const int rla = min(ra, rows - 1), rlb = min(ra + 1, rows - 1);      // rows in the chunk (rows >= 1)
    const float* wa = wf + (size_t)rla * n;
    const float* wb = wf + (size_t)rlb * n;
    const unsigned char* pa = pup + (size_t)rla * n;
    const unsigned char* pb = pup + (size_t)rlb * n;
    float2 x[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        if (n1 < WLO || n1 > WHI) {
            x[n1] = make_float2(0.f, 0.f);
            continue;
        }
        const int qc = N2 * n1 + t - p0;
        const bool in = active && qc >= 0 && qc < n;
        const int qs = min(max(qc, 0), n - 1);
        const unsigned char ma = pa[qs], mb = pb[qs];
        const float va = wa[qs], vb = wb[qs];
        x[n1] = make_float2(in && ma ? va : 0.f, in && has_b && mb ? vb : 0.f);
    }
    if (mode != 0) {
        // partial moments (sum v, sum x v, sum y v) of the chunk, coordinates about the pupil centre
        const float half = 0.5f * (float)(n - 1);
        const float xa = (float)(r0 + ra) - half, xb = xa + 1.f;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const float y = (float)(N2 * n1 + t - p0) - half;
            const float s = x[n1].x + x[n1].y;
            m0 += s;
            m1 = fmaf(xa, x[n1].x, fmaf(xb, x[n1].y, m1));
            m2 = fmaf(y, s, m2);
        }
        for (int o = 32; o > 0; o >>= 1) {
            m0 += __shfl_xor(m0, o, 64);
            m1 += __shfl_xor(m1, o, 64);
            m2 += __shfl_xor(m2, o, 64);
        }
        const int wave = tid / 64, nw = (nthr + 63) / 64;
        if ((tid & 63) == 0) {
            red[3 * wave + 0] = m0;
            red[3 * wave + 1] = m1;
            red[3 * wave + 2] = m2;
        }
        __syncthreads();
        if (tid == 0) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
            for (int w = 0; w < nw; ++w) {
                s0 += red[3 * w + 0];
                s1 += red[3 * w + 1];
                s2 += red[3 * w + 2];
            }
            // the chunk's share of the plane coefficients (the fit is linear in the data)
            a.part[((size_t)f * a.J + a.slot[star]) * gridDim.x + chunk] =
                make_float2(a.tt_b[0] * s0 + a.tt_b[1] * s1 + a.tt_b[2] * s2,
                            a.tt_c[0] * s0 + a.tt_c[1] * s1 + a.tt_c[2] * s2);
        }
    }
    if (mode == 2) return;          // natural star of a mixed asterism: only its plane is used

    // the team's own region (the moment reduction above uses another part of LDS)
    if (active) fft_pass1_regs<M, -1>(t, xch, twr, x);
    team_sync();                    // the team's own region
    float2 zr[N1 / T][N2];
    if (active) fft_pass2_load<M>(t, xch, zr);
    team_sync();                    // the team's own region
    if (active) fft_pass2_regs<M, -1>(t, zr, [&](int k, float2 v) { xch[k] = v; });
    __syncthreads();

    // separate the two real rows of each pair, A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i,
    // and write the half spectrum k < M/2, rows contiguous; thread -> (k, pair) over a power-of-two
    // number of pair slots
    int lg = 0;
    while ((1 << lg) < nteams) ++lg;
    const int npair = (rows + 1) / 2;
    float2* Rb = a.R + ((size_t)f * a.J + a.slot[star]) * (size_t)Kh * n + r0;
    for (int idx = tid; idx < (KC << lg); idx += nthr) {
        const int k = idx >> lg;
        const int pr = idx & ((1 << lg) - 1);
        if (pr < npair) {
            const float2* z = smem + pr * TS;
            const float2 zk = z[k];
            const float2 zm = cconj(z[(M - k) & (M - 1)]);
            float2* dst = Rb + (size_t)k * n + 2 * pr;
            dst[0] = cscale(cadd(zk, zm), 0.5f);
            if (2 * pr + 1 < rows) {
                const float2 d = csub(zk, zm);
                dst[1] = make_float2(0.5f * d.y, -0.5f * d.x);
            }
        }
    }
}

// One wavefront per (frame, slot): the parts of its plane coefficients added.  Lane q adds chunks q,
// q + 64, ... (all loads in flight together), then a fixed shuffle tree sums the lanes, so every call adds
// in the same order.
__global__ __launch_bounds__(256) void plane_kernel(PlaneKArgs a) {
    const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= a.count) return;                       // whole wavefronts leave together
    const float2* pt = a.part + (size_t)i * a.nchunk;
    float2 s = make_float2(0.f, 0.f);
    for (int q = lane; q < a.nchunk; q += 64) {
        const float2 v = pt[q];
        s.x += v.x;
        s.y += v.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        s.x += __shfl_xor(s.x, o, 64);
        s.y += __shfl_xor(s.y, o, 64);
    }
    if (lane == 0) a.planes[i] = s;
}

hipError_t launch_planes(const PlaneKArgs& a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(plane_kernel, dim3((a.count + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int M, int NN>
static hipError_t launch_rows_t(const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s) {
    constexpr int T = FftShape<M>::T;
    const size_t lds = rows_lds_bytes(M, a.n, teams);
    allow_large_lds(reinterpret_cast<const void*>(&rows_kernel<M, NN>));
    const int threads = ((teams * T + 63) / 64) * 64;       // whole wavefronts (the reduction uses all lanes)
    hipLaunchKernelGGL((rows_kernel<M, NN>), dim3(nchunk, a.J, frames), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// pupil sizes of the configured workloads get a compile-time kernel (n = 69 at M = 256, 41 at 128, 33 at 64)
hipError_t launch_rows(int M, const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s) {
    switch (M) {
        case 32: return launch_rows_t<32, 0>(a, frames, nchunk, teams, s);
        case 64: return a.n == 33 ? launch_rows_t<64, 33>(a, frames, nchunk, teams, s)
                                  : launch_rows_t<64, 0>(a, frames, nchunk, teams, s);
        case 128: return a.n == 41 ? launch_rows_t<128, 41>(a, frames, nchunk, teams, s)
                                   : launch_rows_t<128, 0>(a, frames, nchunk, teams, s);
        case 256: return a.n == 69 ? launch_rows_t<256, 69>(a, frames, nchunk, teams, s)
                                   : launch_rows_t<256, 0>(a, frames, nchunk, teams, s);
        default: return hipErrorInvalidValue;
    }
}

size_t rows_lds_bytes(int M, int n, int teams) {
    (void)n;
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    return (size_t)teams * (N1 * (N2 + 1) + 2) * sizeof(float2) + 64 * sizeof(float);
}

}  // namespace safr
