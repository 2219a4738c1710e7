// Natural-star basis images of a mixed asterism (split tomography, Sec. 3.3), FP64.
//
// The natural-star group sees only the least-squares tip/tilt plane b_g x + c_g y
// of each of its wavefronts over the pupil.  Alg. 1 is linear, so its layers on
// the laser-star grids are
//     N_l = resample_l( IDFT2( sum_g B_lg (b_g X + c_g Y) ) )
//         = sum_g b_g P[l][2g] + c_g P[l][2g + 1],
//     P[l][2g]     = resample_l( IDFT2( B_lg X ) ),
//     P[l][2g + 1] = resample_l( IDFT2( B_lg Y ) ),
// with X, Y the DFT2 of x * pupil, y * pupil zero-extended, IDFT2 including the
// 1/M^2 of Sec. 3.2 and resample_l the periodic bilinear sampling at fractional
// index u = c_l (p - M/2) + M/2 on both axes.  The hard-real-time step then adds
// these 2 G_ngs fixed images with the frame's plane coefficients instead of
// transforming the natural-star layers.
//
//   basis_cols_kernel:  T[b][k][p] = sum_j S_b(j, k) e^(+2 pi i j p / M),
//                       S_b = B[k][l][g][j] * (X or Y)[k][j] on the half spectrum;
//   basis_rows_kernel:  E[b][p][q] = M^-2 (T[b][0][p] + T[b][M/2][p] (-1)^q
//                       + 2 Re sum_{0 < k < M/2} T[b][k][p] e^(+2 pi i k q / M))
//                       (real parts of T at k = 0 and M/2: the spectrum is Hermitian);
//   basis_resample_kernel: P[l][i][p][q] (FP32) from E.
// Twiddles come from an FP64 table of e^(2 pi i e / M), indexed by (j p) mod M.
#include "safr_internal.h"

namespace safr {

namespace {

__global__ void basis_cols_kernel(BasisArgs a) {
    const int M = a.M, Kh = M / 2 + 1;
    const size_t total = (size_t)a.L * a.G * 2 * Kh * M;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int p = (int)(idx % M);
    const int k = (int)((idx / M) % Kh);
    const int b = (int)(idx / ((size_t)M * Kh));       // b = (l * G + g) * 2 + axis
    const int axis = b & 1, g = (b >> 1) % a.G, l = (b >> 1) / a.G;
    const double2* H = (axis == 0 ? a.X : a.Y) + (size_t)k * M;
    const double2* Bk = a.B64 + (((size_t)k * a.L + l) * a.G + g) * M;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < M; ++j) {
        const double2 bv = Bk[j], hv = H[j];
        const double vr = bv.x * hv.x - bv.y * hv.y, vi = bv.x * hv.y + bv.y * hv.x;
        const double2 w = a.tw64[(j * p) & (M - 1)];
        sr += vr * w.x - vi * w.y;
        si += vr * w.y + vi * w.x;
    }
    a.T[idx] = make_double2(sr, si);
}

__global__ void basis_rows_kernel(BasisArgs a) {
    const int M = a.M, Kh = M / 2 + 1;
    const size_t total = (size_t)a.L * a.G * 2 * M * M;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int q = (int)(idx % M);
    const int p = (int)((idx / M) % M);
    const int b = (int)(idx / ((size_t)M * M));
    const double2* Tb = a.T + (size_t)b * Kh * M;
    double s = Tb[p].x + ((q & 1) ? -Tb[(size_t)(M / 2) * M + p].x : Tb[(size_t)(M / 2) * M + p].x);
    for (int k = 1; k < M / 2; ++k) {
        const double2 v = Tb[(size_t)k * M + p];
        const double2 w = a.tw64[(k * q) & (M - 1)];
        s += 2.0 * (v.x * w.x - v.y * w.y);
    }
    a.E[idx] = s / ((double)M * (double)M);
}

__global__ void basis_resample_kernel(BasisArgs a) {
    const int M = a.M;
    const size_t total = (size_t)a.L * a.G * 2 * M * M;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int q = (int)(idx % M);
    const int p = (int)((idx / M) % M);
    const int b = (int)(idx / ((size_t)M * M));
    const int l = (b >> 1) / a.G;
    const double c = a.c[l], hm = 0.5 * M;
    const double u = c * (p - hm) + hm, w = c * (q - hm) + hm;
    const double fu0 = floor(u), fw0 = floor(w);
    const double fu = u - fu0, fw = w - fw0;
    const int i0 = ((int)fu0) & (M - 1), i1 = (i0 + 1) & (M - 1);
    const int j0 = ((int)fw0) & (M - 1), j1 = (j0 + 1) & (M - 1);
    const double* Eb = a.E + (size_t)b * M * M;
    const double top = (1.0 - fw) * Eb[(size_t)i0 * M + j0] + fw * Eb[(size_t)i0 * M + j1];
    const double bot = (1.0 - fw) * Eb[(size_t)i1 * M + j0] + fw * Eb[(size_t)i1 * M + j1];
    // P layout [l][i][p][q] with i = 2 g + axis, which is the order of b within a layer
    a.P[idx] = (float)((1.0 - fu) * top + fu * bot);
}

}  // namespace

hipError_t launch_ngs_basis(const BasisArgs& a, hipStream_t s) {
    const int Kh = a.M / 2 + 1;
    const size_t n1 = (size_t)a.L * a.G * 2 * Kh * a.M;
    const size_t n2 = (size_t)a.L * a.G * 2 * a.M * a.M;
    hipLaunchKernelGGL(basis_cols_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(basis_rows_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(basis_resample_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace safr
