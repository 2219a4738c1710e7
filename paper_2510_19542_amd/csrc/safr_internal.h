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

// The star group the column kernels transform: all stars of a single-kind
// asterism (mode 0), or the laser stars of a mixed one (mode 1: tip/tilt plane
// removed).  The natural stars of a mixed asterism enter through precomputed
// basis images in the output pass (Sec. 3.3).  Per-star data of a call (row
// spectra, plane coefficients) is stored in group order, the transformed group's
// stars in slots 0 .. G - 1, so the column kernels address member g directly.
struct GroupArgs {
    int G;                  // stars in the group
    int mode;               // 0 plain, 1 remove the tip/tilt plane
};

// Row pass (forward): pupil mask, tip/tilt moments and the R2C FFT of the n
// nonzero rows of each zero-extended wavefront.  R layout [f][slot][k][n] with
// star g's spectra in its group slot slot[g] (the natural stars of a mixed
// asterism, which are not transformed, leave their slots unwritten).
struct RowArgs {
    const float* wf;            // [F][J][n][n]
    float2* R;                  // [F][J][Kh][n]
    float2* part;               // [F][J][nchunk] tip/tilt plane coefficients of each row chunk, group order
    float tt_b[3], tt_c[3];     // rows 1 and 2 of the inverse normal matrix of the plane fit of [1, x, y]
    const unsigned char* pupil; // [n][n]
    const float2* tw;           // (cos, sin)(2 pi e / M), e < M
    int n, J, p0, rows_per_block;
    int slot[kMaxJ];            // group slot of star g
    int tt_mode[kMaxJ];         // star g: 0 none, 1 remove tip/tilt, 2 plane only (moments, no transform)
};

// Sum over layers of the commands `lay` ([L][M][M]) sampled by periodic bilinear interpolation at
// (u0 + m i, v0 + m j) for tab[l] = (m, u0, v0, -): the layered operator of Sec. 2 along one line of
// sight at pixel (i, j).  M a power of two; LC > 0 fixes L at compile time (all samples issued at once).
template <int LC>
__device__ __forceinline__ float los_sum(const float* __restrict__ lay, const float4* __restrict__ tab, int L, int M,
                                         int i, int j) {
    const int mask = M - 1;
    const int nl = LC > 0 ? LC : L;
    float acc = 0.f;
#pragma unroll
    for (int l = 0; l < (LC > 0 ? LC : kMaxL); ++l) {
        if (LC == 0 && l >= nl) break;
        const float4 t = tab[l];
        const float u = fmaf(t.x, (float)i, t.y);
        const float w = fmaf(t.x, (float)j, t.z);
        const float fu0 = floorf(u), fw0 = floorf(w);
        const float fu = u - fu0, fw = w - fw0;
        const int i0 = (int)fu0 & mask, j0 = (int)fw0 & mask;
        const int i1 = (i0 + 1) & mask, j1 = (j0 + 1) & mask;
        const float* X = lay + (size_t)l * M * M;
        const float x00 = X[i0 * M + j0], x01 = X[i0 * M + j1];
        const float x10 = X[i1 * M + j0], x11 = X[i1 * M + j1];
        acc += (1.f - fu) * ((1.f - fw) * x00 + fw * x01) + fu * ((1.f - fw) * x10 + fw * x11);
    }
    return acc;
}

// Layer spectra after the inverse column transforms, in row tiles of 8:
// C[f][l][p / 8][k][p % 8] (float2), so that a tile of 8 rows is contiguous.
__host__ __device__ inline size_t c_index(int f, int l, int L, int M, int k, int p) {
    return ((((size_t)f * L + l) * (M / 8) + (p >> 3)) * (M / 2 + 1) + k) * 8 + (p & 7);
}

// Column pass: column FFT of the group's spectra, per-frequency apply of B,
// inverse column FFT of the L layer spectra into C.
struct ColArgs {
    const float2* R;            // [F][J][Kh][n], group order
    const float2* B;            // [column block][l][g][column in block][j] (FP32 complex)
    float2* C;                  // see c_index
    const float2* tw;
    const float2* planes;       // tip/tilt plane coefficients per (frame, group slot), see PlaneArgs
    int plane_nch;              // parts per plane (row chunks, or 1 when already added)
    const float2* Xh;           // DFT2 of x * pupil, [Kh][M]
    const float2* Yh;           // DFT2 of y * pupil, [Kh][M]
    GroupArgs grp;
    int n, J, L, p0, frames, frames_per_block;
    int prefetch;               // 1 = compile-time shape (d in registers, inputs prefetched), when available
    const float2* Bm;           // B in the matrix-core lane layout (see pack_mfma_b), or nullptr
};

// B of the transformed group in the lane layout of the matrix-core apply (v_mfma_f32_4x4x1f32: 16 blocks of
// 4 x 4, K = 1): per column block kb, group q of 16 (column, frequency) pairs, star g and layer block lb, 64
// float2 where lane i holds B[l = 4 lb + i % 4][g] of pair 16 q + i / 4 (zero for l >= L), from the FP32
// column-pass layout.  Complex count: column blocks x 16 x G x ceil(L / 4) x 64.
size_t mfma_b_count(int M, int L, int G);
hipError_t launch_pack_mfma_b(int M, int L, int G, const float2* B32, float2* Bm, hipStream_t s);

// Output pass: C2R row transforms, scaling by 1/M^2, and (mixed asterisms) the
// natural-star layers from the basis images.
struct OutArgs {
    const float2* C;            // see c_index
    float* out;                 // [F][L][M][M]
    const float2* tw;
    const float* P;             // [L][nb][M][M] natural-star basis images (mixed asterisms)
    const float2* planes;       // tip/tilt plane coefficients per (frame, group slot), see PlaneArgs
    int plane_nch;              // parts per plane (row chunks, or 1 when already added)
    int ngs_base;               // group slot of the first natural star (the laser group's size)
    int nb;                     // 2 x natural stars (0: no natural-star part)
    int L, J, frames, frames_per_block;
    const float* prev;          // integrator (Alg. 3): out = (1 - gain) prev + gain layers; nullptr = plain
    float gain;
};

// Pseudo-open-loop data (Alg. 3): out = pupil .* (wf + weight * A(layers)), A sampled bilinearly along
// each star's line of sight.  tab[g][l] = (m, u0, v0, 0): pupil pixel (i, j) of star g crosses output
// layer l at the fractional grid index (u0 + m i, v0 + m j).
struct PolcArgs {
    const float* wf;            // [F][J][n][n]
    const float* layers;        // [F][L][M][M]
    float* out;                 // [F][J][n][n]
    const unsigned char* pupil; // [n][n]
    const float4* tab;          // [J][L]
    float weight;
    int n, M, J, L;
};
hipError_t launch_polc(const PolcArgs& a, int frames, hipStream_t s);

// Strehl estimate (Marechal): residual phase open_loop - A_theta(layers) over the pupil for science
// directions theta (cone coefficient 1), its piston-removed variance, exp(-variance).
constexpr int kMaxDirs = 32;
struct StrehlArgs {
    const float* open_loop;     // [F][D][n][n]
    const float* layers;        // [F][L][M][M]
    float* sr;                  // [F][D]
    float* var;                 // [F][D] or nullptr
    const unsigned char* pupil; // [n][n]
    float dx[kMaxDirs], dy[kMaxDirs];
    float m[kMaxL];             // 1 / c_l: science lines of sight on the output grids
    float base[kMaxL];          // m_l (p0 - M/2) + M/2
    float hs[kMaxL];            // h_l / (c_l pitch): layer pixels per radian of direction
    float scale2;               // (phase unit -> rad)^2
    float* part;                // [F][D][chunks][3] per-chunk (count, mean, M2) of the residual
    int n, M, L, D;
};
int strehl_chunks(int n);

// Debug input check: *first = min(*first, frame) for every frame with a non-finite value (pupil != nullptr:
// only where pupil[e % pix] is set; per_frame a multiple of pix).
hipError_t launch_finite_check(const float* x, const unsigned char* pupil, int pix, int per_frame, int frames,
                               int* first, hipStream_t s);       // pupil chunks (256 pixels each) per frame and direction
hipError_t launch_strehl(const StrehlArgs& a, int frames, hipStream_t s);
// Deadline monitor of the closed-loop step: stats [steps, misses, last, max, start] in wall-clock ticks.
hipError_t launch_deadline_start(unsigned long long* stats, hipStream_t s);
hipError_t launch_deadline_end(unsigned long long* stats, unsigned long long period_ticks, hipStream_t s);

// BF16 hi/lo split apply on matrix cores (batched path).
struct MfmaArgs {
    const float2* R;
    const uint16_t* Apack;      // packed real-split B tiles, hi and lo (bf16 bit patterns)
    float2* C;
    const float2* tw;
    const float2* planes;       // tip/tilt plane coefficients per (frame, group slot), see PlaneArgs
    int plane_nch;              // parts per plane (row chunks, or 1 when already added)
    const float2* Xh;
    const float2* Yh;
    GroupArgs grp;
    int n, J, L, p0, frames;
    int lt;                     // layers per tile
    int ntile;                  // layer tiles
    int ppm;                    // frequencies packed per matrix op
};

// Natural-star basis images (FP64 precompute of a mixed asterism).
struct BasisArgs {
    int M, L, G;                // G natural stars
    double c[kMaxL];            // laser-grid cone coefficients (resample positions)
    const double2* B64;         // natural group's B, [Kh][L][G][M]
    const double2* X;           // DFT2 of x * pupil, [Kh][M]
    const double2* Y;           // DFT2 of y * pupil, [Kh][M]
    const double2* tw64;        // e^(2 pi i e / M), e < M
    double2* T;                 // scratch [L * G * 2][Kh][M]
    double* E;                  // scratch [L * G * 2][M][M]
    float* P;                   // [L][2 G][M][M]
};

// Tip/tilt plane coefficients (b, c) of every (frame, star) of a call (Sec. 3.3: the least-squares plane).
// The fit is linear in the wavefront, so each block of the row pass writes the coefficients of its own
// chunk of rows, part[f][slot][chunk] (float2, nch chunks), and a pass needing a plane adds its nch parts.
// Stars are in group order: the laser (or only) group's stars in slots 0 .. G0 - 1 and the natural stars
// of a mixed asterism after them, so a pass reads its group's coefficients without looking up star indices
// (a dependent load would make it wait for every earlier memory operation).  With more than kPlaneLanes
// chunks, plane_kernel adds them first and the passes read its sums with nch = 1.
//
// A pass needing the planes of `count` pairs, pair i = (frame f0 + i / per, group slot base + i % per),
// frames at or beyond fend using fend - 1, requests them early with plane_fetch (kPlaneLanes consecutive
// threads per pair, one chunk each, PMAX rounds of blockDim / kPlaneLanes pairs in registers) and adds
// and stores them to out[i] (LDS) with plane_put (a fixed lane tree: ((p0 + p1) + (p2 + p3)) +
// ((p4 + p5) + (p6 + p7)), absent parts zero); pairs beyond PMAX rounds are added there directly, in the
// same order.  Every thread of the block calls both with the same arguments.
constexpr int kPlaneLanes = 8;

struct PlaneArgs {
    const float2* part;
    int nch, J, per, f0, fend, count, base;
};

__device__ inline const float2* plane_src(const PlaneArgs& p, int i) {
    const int f = min(p.f0 + i / p.per, p.fend - 1);
    return p.part + ((size_t)f * p.J + p.base + i % p.per) * p.nch;
}

__device__ inline float2 plane_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

__device__ inline float2 plane_at(const PlaneArgs& p, int i) {
    const float2* src = plane_src(p, i);
    float2 v[kPlaneLanes];
#pragma unroll
    for (int c = 0; c < kPlaneLanes; ++c) v[c] = c < p.nch ? src[c] : make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 1; w < kPlaneLanes; w *= 2)
#pragma unroll
        for (int c = 0; c < kPlaneLanes; c += 2 * w) v[c] = plane_add(v[c], v[c + w]);
    return v[0];
}

template <int PMAX>
__device__ inline void plane_fetch(const PlaneArgs& p, float2 (&v)[PMAX]) {
    const int c = (int)threadIdx.x % kPlaneLanes, per_round = (int)blockDim.x / kPlaneLanes;
#pragma unroll
    for (int u = 0; u < PMAX; ++u) {
        const int i = (int)threadIdx.x / kPlaneLanes + u * per_round;
        // always issued (count, nch >= 1): no branch; lanes without a part are zeroed in plane_put, so
        // nothing here waits for the load
        v[u] = plane_src(p, min(i, p.count - 1))[min(c, p.nch - 1)];
    }
}

// the value of another lane of the same row of 16 (data-parallel-primitive lane move, no LDS round trip)
template <int CTRL>
__device__ inline float2 plane_dpp(float2 v) {
    return make_float2(__int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v.x), CTRL, 0xF, 0xF, false)),
                       __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v.y), CTRL, 0xF, 0xF, false)));
}

// REM: pairs beyond PMAX rounds may occur (otherwise the caller guarantees count <= PMAX blockDim / 8)
template <int PMAX, bool REM = true>
__device__ inline void plane_put(const PlaneArgs& p, const float2 (&v)[PMAX], float2* out) {
    static_assert(kPlaneLanes == 8, "the lane tree below adds 8 lanes");
    const int c = (int)threadIdx.x % kPlaneLanes, per_round = (int)blockDim.x / kPlaneLanes;
#pragma unroll
    for (int u = 0; u < PMAX; ++u) {
        const int i = (int)threadIdx.x / kPlaneLanes + u * per_round;
        float2 s = i < p.count && c < p.nch ? v[u] : make_float2(0.f, 0.f);
        s = plane_add(s, plane_dpp<0xB1>(s));       // lanes 1 0 3 2 of each quad: pairs of parts
        s = plane_add(s, plane_dpp<0x4E>(s));       // lanes 2 3 0 1: the quad's sum in all its lanes
        s = plane_add(s, plane_dpp<0x141>(s));      // lane 7 - i of each 8: the other quad's sum
        if (c == 0 && i < p.count) out[i] = s;
    }
    if constexpr (REM)
        for (int i = (int)threadIdx.x + PMAX * per_round; i < p.count; i += blockDim.x) out[i] = plane_at(p, i);
}

// More than kPlaneLanes row chunks: the parts of `count` = F x J (frame, slot) pairs added in chunk order
// into planes[f][slot] (the passes then read them with nch = 1).
struct PlaneKArgs {
    const float2* part;         // [F][J][nchunk] in group order
    float2* planes;             // [F][J] in group order
    int nchunk, count;
};
hipError_t launch_planes(const PlaneKArgs& a, hipStream_t s);

// Lets a kernel use up to the full 160 KiB of LDS of a gfx950 compute unit (once per kernel).
inline void allow_large_lds(const void* kernel) {
    static thread_local const void* done[64];
    static thread_local int ndone = 0;
    for (int i = 0; i < ndone; ++i)
        if (done[i] == kernel) return;
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    if (ndone < 64) done[ndone++] = kernel;
}

// The whole step of one frame per block for the small configured geometry (see k_frame.hip): wavefronts
// [F][4][33][33], layers [F][L][64][64], B of the one group in the column pass's layout.
struct FrameArgs {
    const float* wf;
    const unsigned char* pupil; // [n][n]
    const float2* tw;           // (cos, sin)(2 pi e / M), e < M
    const float2* B;            // [k / 4][l][g][k % 4][j] (FP32, 1/M^2 included)
    float* out;
    const float* prev;          // integrator (Alg. 3): out = (1 - gain) prev + gain layers; nullptr = plain
    float gain;
    int frames;
};
bool frame_shape(int M, int n, int G, int L, int mode);
size_t frame_lds_bytes();
hipError_t launch_frame(const FrameArgs& a, int L, hipStream_t s);

// Launchers (defined in the .hip files); return hipSuccess or the launch error.
hipError_t launch_rows(int M, const RowArgs& a, int frames, int nchunk, int teams, hipStream_t s);
hipError_t launch_cols(int M, const ColArgs& a, int frames_together, int frames, hipStream_t s);
bool cols_fixed_shape(int M, int L, int G, int mode);
hipError_t launch_out(int M, const OutArgs& a, int rows_per_block, int frames, hipStream_t s);
hipError_t launch_ngs_basis(const BasisArgs& a, hipStream_t s);
bool out_rows_supported(int M, int rows_per_block);
int out_frames_per_iter(int M, int rows_per_block);
hipError_t launch_cols_mfma(int M, const MfmaArgs& a, int frames, int frames_per_block, hipStream_t s);
size_t rows_lds_bytes(int M, int n, int teams);
size_t out_lds_bytes(int M, int rows_per_block, int nb);
size_t mfma_lds_bytes(int M, int frames_per_block, int gmax, int L);
size_t cols_lds_bytes(int M, int G, int L, int frames_together, bool fixed, bool mf = false);

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
    int tsvd;         // 1 = truncated SVD instead of Tikhonov (no learned filter)
    const double* aw; // [M][M] per-frequency multipliers of alpha, or nullptr
};
hipError_t launch_svd(const PrecompArgs& a, hipStream_t s);
hipError_t launch_assemble(const PrecompArgs& a, hipStream_t s);
hipError_t launch_mlp_infer(const float* params, const float* feats, float* phi, int rows, float log10_noise,
                            hipStream_t s);
safr_status set_error(safr_status st, const char* msg);
hipError_t launch_pack_bf16(int M, int L, int G, const float2* B32, uint16_t* Apack, int lt, int ntile,
                            int ppm, hipStream_t s);

}  // namespace safr
