// Debug check of a call's inputs: the smallest frame index holding a non-finite
// value (at a pupil pixel for wavefronts, anywhere for layer-shaped inputs).
#include "safr_internal.h"

namespace safr {

__global__ void __launch_bounds__(256) finite_check_kernel(const float* x, const unsigned char* pupil, int pix,
                                                           int per_frame, size_t total, int* first) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const int e = (int)(i % (size_t)per_frame);
        if (pupil && !pupil[e % pix]) continue;
        if (!isfinite(x[i])) atomicMin(first, (int)(i / (size_t)per_frame));
    }
}

hipError_t launch_finite_check(const float* x, const unsigned char* pupil, int pix, int per_frame, int frames,
                               int* first, hipStream_t s) {
    if (!x || !first || pix < 1 || per_frame < 1 || per_frame % pix || frames < 1) return hipErrorInvalidValue;
    const size_t total = (size_t)per_frame * frames;
    const size_t want = (total + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(finite_check_kernel, dim3(blocks), dim3(256), 0, s, x, pupil, pix, per_frame, total, first);
    return hipGetLastError();
}

}  // namespace safr
