// Internal definitions shared by the host side of the library and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/safr.h"

namespace safr {

constexpr int kMaxG = SAFR_MAX_STARS_PER_GROUP;
constexpr int kMaxL = SAFR_MAX_LAYERS;
constexpr int kMaxJ = 2 * kMaxG;
constexpr double kSqrtEps = 1.4901161193847656e-08;   // 2^-26: the learned filter's relative cutoff

// Per-group description passed by value to the column kernel.
struct GroupArgs {
    int G;                  // stars in the group
    int mode;               // 0 plain, 1 remove the tip/tilt plane, 2 keep only the plane
    int star[kMaxG];        // star index of member g
    size_t b_off;           // offset of the group's B in the FP32 B array (complex elements)
};

struct GroupSet {
    int count;
    GroupArgs g[2];
};

// Row pass (forward): pupil mask, tip/tilt handling and the R2C FFT of the n
// nonzero rows of each zero-extended wavefront.  R layout [f][star][k][n].
struct RowArgs {
    const float* wf;            // [F][J][n][n]
    float2* R;                  // [F][J][Kh][n]
    float* mom;                 // [F][J][nchunk][4] partial moments (sum v, sum x v, sum y v, 0)
    const unsigned char* pupil; // [n][n]
    const int* tt_mode;         // [J]: 0 none, 1 remove tip/tilt, 2 keep tip/tilt
    const float2* tw;           // (cos, sin)(2 pi e / M), e < M
    int n, J, p0, rows_per_block;
};

// Column pass: column FFT of the J spectra, per-frequency apply of B, inverse
// column FFT of the L layer spectra.  C layout [f][group][l][k][p].
struct ColArgs {
    const float2* R;            // [F][J][Kh][n]
    const float2* B;            // per group: [column block][l][g][column in block][j] (FP32 complex)
    float2* C;                  // [F][groups][L][Kh][M]
    const float2* tw;
    const float* mom;           // partial moments from the row pass
    const float2* Xh;           // DFT2 of x * pupil, [Kh][M]
    const float2* Yh;           // DFT2 of y * pupil, [Kh][M]
    float tt_b[3], tt_c[3];     // rows 1 and 2 of the inverse normal matrix of the fit of [1, x, y]
    GroupSet groups;
    int n, J, L, p0, frames, frames_per_block, nchunk, gmax;
    int prefetch;               // 1 = keep the block's B in registers (L * G <= 64)
};

// Output pass: C2R row transforms, scaling by 1/M^2, and (mixed asterisms) the
// bilinear resample-and-add of the natural-star layers.
struct OutArgs {
    const float2* C;            // [F][groups][L][Kh][M]
    float* out;                 // [F][L][M][M]
    const float2* tw;
    float c[kMaxL];             // output-grid cone coefficients (resample positions)
    int L, groups, mixed, rows_per_block, ngs_group;
};

// BF16 hi/lo split apply on matrix cores (batched path).
struct MfmaArgs {
    const float2* R;
    const uint16_t* Apack;      // packed real-split B tiles, hi and lo (bf16 bit patterns)
    float2* C;
    const float2* tw;
    const float* mom;
    const float2* Xh;
    const float2* Yh;
    float tt_b[3], tt_c[3];
    GroupSet groups;
    size_t a_off[2];            // per-group offset into Apack (uint16 elements)
    int n, J, L, p0, frames, nchunk, gmax;
    int lt[2];                  // layers per tile (per group)
    int ntile[2];               // layer tiles per group
    int ppm[2];                 // frequencies packed per matrix op (per group)
};

// Lets a kernel use up to the full 160 KiB of LDS of a gfx950 compute unit (once per kernel).
inline void allow_large_lds(const void* kernel) {
    static thread_local const void* done[64];
    static thread_local int ndone = 0;
    for (int i = 0; i < ndone; ++i)
        if (done[i] == kernel) return;
    hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    if (ndone < 64) done[ndone++] = kernel;
}

// Launchers (defined in the .hip files); return hipSuccess or the launch error.
hipError_t launch_rows(int M, const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s);
hipError_t launch_cols(int M, const ColArgs& a, int frames, hipStream_t s);
hipError_t launch_out(int M, const OutArgs& a, int frames, hipStream_t s);
hipError_t launch_cols_mfma(int M, const MfmaArgs& a, int frames, int frames_per_block, hipStream_t s);
size_t rows_lds_bytes(int M, int n, int teams);
size_t out_lds_bytes(int M, int rows_per_block, bool mixed);
size_t mfma_lds_bytes(int M, int frames_per_block, int gmax, int L);
size_t cols_lds_bytes(int M, int gmax, int L);

// Precompute (FP64): SVD per half-spectrum frequency and the assembly of B.
struct PrecompArgs {
    int M, G, L;
    double T, beta, alpha;
    double ax[kMaxG], ay[kMaxG];
    double h[kMaxL], c[kMaxL], sqrt_gamma[kMaxL], gamma[kMaxL];
    double2* W;       // [H][R][C] rotated columns (R = max(G,L), C = min(G,L))
    double2* Q;       // [H][C][C] accumulated rotations
    double* sigma;    // [H][C]
    float* feats;     // [H][C][4] network inputs (learned filter)
    float* phi;       // [H][C] network outputs (learned filter), or nullptr for Tikhonov
    double2* B64;     // [Kh][L][G][M] group block
    float2* B32;
    double log10_noise;
    int* bad;         // set to 1 if a non-finite value appears
};
hipError_t launch_svd(const PrecompArgs& a, hipStream_t s);
hipError_t launch_assemble(const PrecompArgs& a, hipStream_t s);
hipError_t launch_mlp_infer(const float* params, const float* feats, float* phi, int rows, float log10_noise,
                            hipStream_t s);
safr_status set_error(safr_status st, const char* msg);
hipError_t launch_pack_bf16(int M, int L, int G, const float2* B32, uint16_t* Apack, int lt, int ntile,
                            int ppm, hipStream_t s);

}  // namespace safr
