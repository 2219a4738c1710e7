// Row pass of the forward 2-D transform (Alg. 1, first loop).
//
// The zero-extended M x M wavefront has only n nonzero rows and columns, so
// only the n pupil rows are transformed; two real rows are packed into one
// complex M-point FFT (z = a + i b) and separated afterwards with
// A[k] = (Z[k] + conj Z[-k]) / 2,  B[k] = (Z[k] - conj Z[-k]) / (2 i).
// Output: R[f][star][k][row] for k = 0..M/2 (half spectrum), rows contiguous so
// the column pass reads each column as one run.
//
// Split tomography (Sec. 3.3) needs the least-squares tip/tilt plane of each
// wavefront over the pupil.  Each block writes the partial moments
// (sum v, sum x v, sum y v) of its own rows; the column pass adds them up and
// removes (laser stars) or keeps only (natural stars) the plane in the Fourier
// domain.  Natural stars of a mixed asterism therefore need no row transform.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

template <int M>
__global__ void rows_kernel(RowArgs a) {
    using S = FftShape<M>;
    constexpr int T = S::T;
    constexpr int Kh = M / 2 + 1;
    constexpr int TL = team_lds<M>();
    extern __shared__ float2 smem[];

    const int n = a.n;
    const int star = blockIdx.y;
    const int f = blockIdx.z;
    const int chunk = blockIdx.x;
    const int r0 = chunk * a.rows_per_block;
    const int rows = min(a.rows_per_block, n - r0);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int team = tid / T;
    const int t = tid % T;
    const int nteams = a.rows_per_block / 2;
    const int mode = a.tt_mode[star];
    const float* wf = a.wf + ((size_t)f * a.J + star) * (size_t)n * n + (size_t)r0 * n;
    const unsigned char* pup = a.pupil + (size_t)r0 * n;

    // LDS: twiddles [M], then one region per team (stride TS, 4 banks apart) that holds in turn the
    // pass-1 -> pass-2 exchange and the packed spectrum, then the staged rows, then 3 floats per
    // wavefront for the moment reduction
    constexpr int TS = TL + 2;
    float2* tws = smem;
    float2* xch = smem + M + team * TS;
    float* vals = reinterpret_cast<float*>(smem + M + nteams * TS);
    float* red = vals + a.rows_per_block * n;

    // stage the block's rows (pupil-masked): all loads of a chunk are issued before any is used
    const float half = 0.5f * (float)(n - 1);
    float m0 = 0.f, m1 = 0.f, m2 = 0.f;
    const int total = rows * n;
    for (int i = tid; i < M; i += nthr) tws[i] = a.tw[i];
    constexpr int CH = 8;
    for (int base = 0; base < total; base += CH * nthr) {
        float v[CH];
        unsigned char m[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int i = base + tid + u * nthr;
            if (i < total) {
                m[u] = pup[i];
                v[u] = wf[i];
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int i = base + tid + u * nthr;
            if (i < total) {
                const float val = m[u] ? v[u] : 0.f;
                vals[i] = val;
                if (mode != 0) {
                    const int pr = i / n;
                    const float x = (float)(r0 + pr) - half;
                    const float y = (float)(i - pr * n) - half;
                    m0 += val;
                    m1 += x * val;
                    m2 += y * val;
                }
            }
        }
    }
    if (mode != 0) {
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
            float* mo = a.mom + (((size_t)f * a.J + star) * gridDim.x + chunk) * 4;
            mo[0] = s0;
            mo[1] = s1;
            mo[2] = s2;
            mo[3] = 0.f;
        }
    }
    if (mode == 2) return;          // natural star of a mixed asterism: only its plane is used
    __syncthreads();

    const int pairs = (rows + 1) / 2;
    float2* Rb = a.R + ((size_t)f * a.J + star) * (size_t)Kh * n;
    for (int base = 0; base < pairs; base += nteams) {
        const int pair = base + team;
        const bool active = team < nteams && pair < pairs;
        const int ra = 2 * pair;
        const bool has_b = active && (ra + 1 < rows);
        if (active) {
            const float* va = vals + ra * n;
            const float* vb = vals + (has_b ? ra + 1 : ra) * n;
            fft_pass1<M, -1>(t, xch, tws, [&](int q) -> float2 {
                const int qc = q - a.p0;
                if (qc < 0 || qc >= n) return make_float2(0.f, 0.f);
                return make_float2(va[qc], has_b ? vb[qc] : 0.f);
            });
        }
        __syncthreads();
        float2 zr[S::N1 / T][S::N2];
        if (active) fft_pass2_load<M>(t, xch, zr);
        __syncthreads();
        if (active) fft_pass2_regs<M, -1>(t, zr, [&](int k, float2 v) { xch[k] = v; });
        __syncthreads();
        // separate the two real rows and write the half spectrum, rows contiguous
        const int nrow = min(2 * nteams, rows - 2 * base);
        for (int idx = tid; idx < Kh * nrow; idx += nthr) {
            const int k = idx / nrow;
            const int r = idx - k * nrow;
            const float2* z = smem + M + (r >> 1) * TS;
            const float2 zk = z[k];
            const float2 zm = cconj(z[(M - k) & (M - 1)]);
            float2 v;
            if ((r & 1) == 0) v = cscale(cadd(zk, zm), 0.5f);
            else {
                const float2 d = csub(zk, zm);
                v = make_float2(0.5f * d.y, -0.5f * d.x);
            }
            Rb[(size_t)k * n + r0 + 2 * base + r] = v;
        }
        __syncthreads();
    }
}

template <int M>
static hipError_t launch_rows_t(const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s) {
    constexpr int T = FftShape<M>::T;
    const size_t lds = rows_lds_bytes(M, a.n, teams);
    allow_large_lds(reinterpret_cast<const void*>(&rows_kernel<M>));
    const int threads = ((teams * T + 63) / 64) * 64;       // whole wavefronts (the reduction uses all lanes)
    hipLaunchKernelGGL(rows_kernel<M>, dim3(nchunk, a.J, frames), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_rows(int M, const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s) {
    switch (M) {
        case 32: return launch_rows_t<32>(a, frames, nchunk, teams, s);
        case 64: return launch_rows_t<64>(a, frames, nchunk, teams, s);
        case 128: return launch_rows_t<128>(a, frames, nchunk, teams, s);
        case 256: return launch_rows_t<256>(a, frames, nchunk, teams, s);
        default: return hipErrorInvalidValue;
    }
}

size_t rows_lds_bytes(int M, int n, int teams) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    return ((size_t)M + (size_t)teams * (N1 * (N2 + 1) + 2)) * sizeof(float2) +
           (size_t)(2 * teams) * n * sizeof(float) + 64 * sizeof(float);
}

}  // namespace safr
