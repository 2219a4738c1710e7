// Debug check of a call's inputs: the smallest frame index holding a non-finite
// value (at a pupil pixel for wavefronts, anywhere for layer-shaped inputs); and the
// deadline monitor of the closed-loop step (a time stamp of the device's constant-rate
// wall clock when the step starts executing, compared with the period when it ends).
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

// st: [0] steps, [1] steps over the period, [2] last duration, [3] longest duration (wall-clock ticks),
// [4] start stamp of the step in progress.  One thread each, in stream order around the step.
__global__ void deadline_start_kernel(unsigned long long* st) { st[4] = wall_clock64(); }

__global__ void deadline_end_kernel(unsigned long long* st, unsigned long long period) {
    const unsigned long long t = wall_clock64() - st[4];
    st[0] += 1;
    if (t > period) st[1] += 1;
    st[2] = t;
    if (t > st[3]) st[3] = t;
}

hipError_t launch_deadline_start(unsigned long long* st, hipStream_t s) {
    hipLaunchKernelGGL(deadline_start_kernel, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_deadline_end(unsigned long long* st, unsigned long long period_ticks, hipStream_t s) {
    hipLaunchKernelGGL(deadline_end_kernel, dim3(1), dim3(1), 0, s, st, period_ticks);
    return hipGetLastError();
}

}  // namespace safr
