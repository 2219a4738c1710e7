// Pseudo-open-loop data for the closed loop (Alg. 3, POLC step).
//
// The mirror commands are layers on the output grids.  For every pupil pixel of
// every guide star the kernel adds, over the layers, the command sampled by
// periodic bilinear interpolation at the point where the star's line of sight
// crosses the layer (the layered tomography operator of Sec. 2), scaled by a
// weight, to the measured wavefront; pixels outside the pupil are written as 0.
// One thread per pupil pixel; the layers (a few MB) are read through L2.
#include "safr_internal.h"

namespace safr {

// L layers as a compile-time count: the 4 L samples of a pixel are all issued before any is used
template <int L>
__global__ void __launch_bounds__(256) polc_kernel(PolcArgs a) {
    const int n = a.n, M = a.M;
    const int g = blockIdx.y, f = blockIdx.z;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n * n) return;
    const size_t o = ((size_t)f * a.J + g) * (size_t)n * n + e;
    float v = 0.f;
    if (a.pupil[e]) {
        const int i = e / n, j = e - (e / n) * n;
        const float acc = los_sum<L>(a.layers + (size_t)f * L * M * M, a.tab + (size_t)g * L, L, M, i, j);
        v = fmaf(a.weight, acc, a.wf[o]);
    }
    a.out[o] = v;
}

namespace {

template <int L>
hipError_t launch_polc_l(const PolcArgs& a, int frames, hipStream_t s) {
    if (a.L != L) return launch_polc_l<L - 1>(a, frames, s);
    const int blocks = (a.n * a.n + 255) / 256;
    hipLaunchKernelGGL(polc_kernel<L>, dim3(blocks, a.J, frames), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <>
hipError_t launch_polc_l<0>(const PolcArgs&, int, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_polc(const PolcArgs& a, int frames, hipStream_t s) {
    if (a.M < 2 || (a.M & (a.M - 1)) || a.n < 1 || a.n > a.M || frames < 1 || frames > 65535 || a.L < 1 ||
        a.L > kMaxL)
        return hipErrorInvalidValue;
    return launch_polc_l<kMaxL>(a, frames, s);
}

}  // namespace safr
