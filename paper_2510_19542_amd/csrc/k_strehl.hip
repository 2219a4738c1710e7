// Strehl ratio by the Marechal approximation (Sec. 4) in science directions.
//
// For each frame and direction theta the residual phase at every pupil pixel is
// the open-loop phase minus the commands sampled along theta (science objects at
// infinity: cone coefficient 1, so on output grid l the pixel (i, j) maps to
// (base_l + m_l i + theta_x hs_l, base_l + m_l j + theta_y hs_l), periodic bilinear
// interpolation).  Its piston-removed variance over the pupil gives the Strehl
// ratio exp(-variance).
//
// Two launches: the partial pass gives every pupil chunk of 256 pixels its own
// block (one pixel per thread, so the chunks of all directions and frames fill
// the chip) and writes the chunk's (count, mean, M2); the merge pass combines a
// (frame, direction)'s chunks with Chan's pairwise formula in an order fixed by the
// chunk count, so the result does not depend on scheduling.
#include "safr_internal.h"

namespace safr {

namespace {

struct Moments {
    float n, mean, m2;
};

__device__ inline Moments merge(Moments a, Moments b) {
    const float n = a.n + b.n;
    if (n == 0.f) return a;
    const float d = b.mean - a.mean;
    const float fb = b.n / n;
    return {n, fmaf(d, fb, a.mean), a.m2 + b.m2 + d * d * a.n * fb};
}

}  // namespace

int strehl_chunks(int n) { return (n * n + 255) / 256; }

template <int L>
__global__ void __launch_bounds__(256) strehl_part_kernel(StrehlArgs a) {
    __shared__ float red[3 * 4];
    const int n = a.n, M = a.M;
    const int c = blockIdx.x, d = blockIdx.y, f = blockIdx.z;
    const int e = c * 256 + threadIdx.x;
    Moments acc = {0.f, 0.f, 0.f};
    if (e < n * n && a.pupil[e]) {
        const int i = e / n, j = e - (e / n) * n;
        // science lines of sight: table entries (m_l, base_l + theta_x hs_l, base_l + theta_y hs_l)
        float4 tab[L];
#pragma unroll
        for (int l = 0; l < L; ++l)
            tab[l] = make_float4(a.m[l], fmaf(a.dx[d], a.hs[l], a.base[l]), fmaf(a.dy[d], a.hs[l], a.base[l]), 0.f);
        const float corr = los_sum<L>(a.layers + (size_t)f * L * M * M, tab, L, M, i, j);
        acc = {1.f, a.open_loop[((size_t)f * a.D + d) * (size_t)n * n + e] - corr, 0.f};
    }
    for (int o = 1; o < 64; o <<= 1) {
        const Moments b = {__shfl_xor(acc.n, o, 64), __shfl_xor(acc.mean, o, 64), __shfl_xor(acc.m2, o, 64)};
        acc = (threadIdx.x & o) ? merge(b, acc) : merge(acc, b);       // both lanes: merge(lower, upper)
    }
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[3 * wave + 0] = acc.n;
        red[3 * wave + 1] = acc.mean;
        red[3 * wave + 2] = acc.m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Moments t = {red[0], red[1], red[2]};
        for (int w = 1; w < 4; ++w) t = merge(t, Moments{red[3 * w], red[3 * w + 1], red[3 * w + 2]});
        float* o = a.part + (((size_t)f * a.D + d) * gridDim.x + c) * 3;
        o[0] = t.n;
        o[1] = t.mean;
        o[2] = t.m2;
    }
}

// one wave per (frame, direction): lane t merges chunks t, t + 64, ... in order, then the lanes merge
// pairwise (lower lane first), so the result is fixed by the chunk count alone
__global__ void __launch_bounds__(64) strehl_merge_kernel(StrehlArgs a, int chunks) {
    const int q = blockIdx.x;                          // q = f * D + d
    const int t = threadIdx.x;
    const float* p = a.part + (size_t)q * chunks * 3;
    Moments acc = {0.f, 0.f, 0.f};
    for (int c = t; c < chunks; c += 64) acc = merge(acc, Moments{p[3 * c], p[3 * c + 1], p[3 * c + 2]});
    for (int o = 1; o < 64; o <<= 1) {
        const Moments b = {__shfl_xor(acc.n, o, 64), __shfl_xor(acc.mean, o, 64), __shfl_xor(acc.m2, o, 64)};
        acc = (t & o) ? merge(b, acc) : merge(acc, b);
    }
    if (t == 0) {
        const float var = acc.n > 0.f ? a.scale2 * (acc.m2 / acc.n) : 0.f;
        a.sr[q] = expf(-var);
        if (a.var) a.var[q] = var;
    }
}

namespace {

template <int L>
hipError_t launch_part_l(const StrehlArgs& a, int chunks, int frames, hipStream_t s) {
    if (a.L != L) return launch_part_l<L - 1>(a, chunks, frames, s);
    hipLaunchKernelGGL(strehl_part_kernel<L>, dim3(chunks, a.D, frames), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <>
hipError_t launch_part_l<0>(const StrehlArgs&, int, int, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_strehl(const StrehlArgs& a, int frames, hipStream_t s) {
    if (a.M < 2 || (a.M & (a.M - 1)) || a.n < 1 || a.n > a.M || a.D < 1 || a.D > kMaxDirs || frames < 1 ||
        frames > 65535 || a.L < 1 || a.L > kMaxL || !a.part)
        return hipErrorInvalidValue;
    const int chunks = strehl_chunks(a.n);
    const hipError_t e = launch_part_l<kMaxL>(a, chunks, frames, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(strehl_merge_kernel, dim3(frames * a.D), dim3(64), 0, s, a, chunks);
    return hipGetLastError();
}

}  // namespace safr
