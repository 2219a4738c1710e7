// Output pass of SAFR's hard-real-time step (Alg. 1, last loop), fused with the
// split-tomography sum (Sec. 3.3):
//   - C2R row transforms of the layer spectra (two real rows packed into one
//     complex inverse FFT); the 1/M^2 of IDFT2 (Sec. 3.2) is already in the FP32 B;
//   - mixed asterisms: the natural-star layers, sum_g b_g P[l][2g] + c_g P[l][2g+1]
//     with the frame's tip/tilt plane coefficients (b_g, c_g) from the row-pass
//     moments and the precomputed basis images P (already resampled onto the
//     laser layer grids), added to every output pixel;
//   - closed loop (Alg. 3): optionally the integrator, out = (1 - gain) prev + gain
//     layer, with prev read at the pixel just before it is written (prev may be out).
//
// One block of 256 threads owns RT rows of one layer and loops over a run of
// frames, NF frames per iteration so that every team of the block transforms
// one row pair: NF = (256 / T) / (RT / 2).  Each team's LDS region holds, in
// turn, its two input rows (Hermitian half spectra), the pass-1 -> pass-2
// exchange and its two output rows; loads of a phase are taken into registers
// and a barrier separates them from the stores that overwrite the region.  The
// next iteration's spectra are requested once the current rows are transformed
// and arrive while the epilogue runs (requested before the transforms, they
// were slower).  The epilogue is pixel-stationary (thread -> 4-pixel groups of
// the block's rows): a group's basis pixels are loaded into registers once per
// block (from L2: the blocks of one row tile are XCD-contiguous) and serve every
// frame of its run.  The kernel runs two wavefronts per SIMD, the occupancy its
// registers allow with the basis pixels held.
//
// C layout (row tiles of 8): C[f][l][p / 8][k][p % 8]; a block's rows of one
// frame are one contiguous run.
#include <type_traits>

#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

#ifndef OUT_WAVES
#define OUT_WAVES 2
#endif

namespace {

// cache policy of the layer stores: non-temporal (2) at device scope (16)
constexpr int kStoreLayers = 2 | 16;

// linear block -> (row block, layer, frame run), XCD-contiguous (blocks are dealt to the 8 XCDs
// round-robin), so the frame runs of one row block and layer share an L2 and its basis pixels
__device__ __forceinline__ bool xcd_work(int nwork, int& w) {
    const int b = blockIdx.x, per = gridDim.x / 8;
    w = (b % 8) * per + b / 8;
    return w < nwork;
}

template <int M, int RT>
struct OutShape {
    static constexpr int T = FftShape<M>::T;
    static constexpr int NTEAM = 256 / T;
    static constexpr int TL = team_lds<M>();
    static constexpr int RS = TL + 2;                               // region stride: 16-byte aligned, 4 banks apart
    static constexpr int Kh = M / 2 + 1;
    static constexpr int TPF = RT / 2;                              // row pairs (teams) per frame
    static constexpr int NF = NTEAM / TPF;                          // frames per iteration
    static constexpr int V4 = RT * M / (4 * 256);                   // 4-pixel groups per thread per frame
    static constexpr int TILE4 = 4 * (M / 2);                       // float4 of one row tile, columns k < M/2
    static constexpr int TPW = (64 / T) / 4;                        // row tiles per wavefront (its teams' row pairs)
    static constexpr int NLD = TPW * TILE4 / 64;                    // float4 loads per lane per iteration
    static_assert(TPF <= NTEAM && NTEAM % TPF == 0, "row pairs must tile the teams");
    static_assert(V4 >= 1 && (RT * M) % 1024 == 0, "at least one 4-pixel group per thread");
    static_assert(2 * Kh <= TL && M <= TL, "a team region holds two rows");
    static_assert(TPW >= 1 && NF * (RT / 8) == 4 * TPW && (TPW * TILE4) % 64 == 0, "a wavefront loads its own tiles");
};

}  // namespace

// NB: natural-star basis images (0: none; 2, 4 or 6: exactly that many; 8: the first 8 of a.nb >= 8, the rest
// re-read per frame).  INTEG: the closed-loop integrator (a.prev is read).
//
// Memory order of an iteration: the vector-memory counter counts loads and stores in issue order, so a
// load can only be waited for together with everything issued before it.  Each iteration therefore
// issues, after its transforms, first the loads it needs itself (its basis pixels), then the next
// iteration's spectra and plane coefficients, and only then its stores; the epilogue waits for the basis
// pixels with the prefetch still in flight, and the next iteration waits for the prefetch without waiting
// for the stores.  Every load is issued unconditionally (inputs past the frame run read the run's last
// frame, which is not stored), so no wait is placed conservatively behind a branch.
template <int M, int RT, int NB, bool INTEG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OUT_WAVES))) void out_kernel(OutArgs a) {
    constexpr bool MIXED = NB > 0;
    constexpr bool TAIL = NB == 8;                                  // more basis images than registers hold
    using S = FftShape<M>;
    using O = OutShape<M, RT>;
    constexpr int T = O::T, RS = O::RS, Kh = O::Kh, NF = O::NF, TPF = O::TPF, V4 = O::V4;
    constexpr int NBR = MIXED ? NB : 1;
    extern __shared__ float2 smem[];

    const int runs = (a.frames + a.frames_per_block - 1) / a.frames_per_block;
    int w;
    if (!xcd_work((M / RT) * a.L * runs, w)) return;               // the whole block leaves before any barrier
    const int frun = w % runs, l = (w / runs) % a.L;
    const int r0 = (w / runs / a.L) * RT;
    const int fbeg = frun * a.frames_per_block;
    const int fend = min(a.frames, fbeg + a.frames_per_block);
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid % T;
    const int L = a.L;
    const int nb = MIXED ? (TAIL ? a.nb : NB) : 0;

    float2* reg = smem + team * RS;                                 // this team's region
    float* coef = reinterpret_cast<float*>(smem + O::NTEAM * RS);   // [NF][nb]

    // spectra of frame f: RT / 8 row tiles of layer l, each Kh * 8 float2 (two float2 per float4); the
    // Nyquist column k = M/2 is neither written by the column pass nor read here
    auto run = [&](int f) {
        return reinterpret_cast<const float4*>(a.C + (((size_t)f * L + l) * (M / 8) + r0 / 8) * Kh * 8);
    };
    // each wavefront loads the row tiles of its own teams (tile = 4 teams = 8 rows of one frame; tile
    // index fi * (RT / 8) + pb), so the spectra it stashes are read by its own teams only
    const int wave = tid >> 6, lane = tid & 63;
    float4 ld[O::NLD];
    auto issue = [&](int fi0) {
#pragma unroll
        for (int i = 0; i < O::NLD; ++i) {
            const int e = lane + 64 * i;
            const int tile = wave * O::TPW + e / O::TILE4, s4 = e % O::TILE4;
            const int fi = tile / (RT / 8), pb = tile % (RT / 8);
            ld[i] = run(min(fi0 + fi, fend - 1))[pb * 4 * Kh + s4];
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < O::NLD; ++i) {
            const int e = lane + 64 * i;
            // float4 s4 of the tile: column k = s4 / 4, rows 2 (s4 % 4) and 2 (s4 % 4) + 1 of the tile
            const int tile = wave * O::TPW + e / O::TILE4, s4 = e % O::TILE4;
            const int k = s4 >> 2;
            float2* dst = smem + (tile * 4 + (s4 & 3)) * RS;
            dst[k] = make_float2(ld[i].x, ld[i].y);
            dst[Kh + k] = make_float2(ld[i].z, ld[i].w);
        }
    };
    // natural stars' plane coefficients (b_g, c_g) of an iteration's frames, [NF][ng] as float2
    auto planes_of = [&](int f0) {
        return PlaneArgs{a.planes, a.plane_nch, a.J, nb / 2, f0, fend, min(NF, fend - f0) * (nb / 2), a.ngs_base};
    };

    // plane lane rounds: every pair in registers unless the basis count is only known at run time
    constexpr int PR = TAIL || !MIXED ? 1 : (NF * (NB / 2) + 256 / kPlaneLanes - 1) / (256 / kPlaneLanes);
    float2 twr[S::N1];                                              // this thread's pass-1 twiddles
    load_pass1_twiddles<M>(a.tw, t, twr);
    issue(fbeg);
    float2 pl[PR];
    if constexpr (MIXED) plane_fetch<PR>(planes_of(fbeg), pl);
    // the block's basis pixels (its rows, every frame): loaded once, before any store
    float4 pv[V4][NBR];
    if constexpr (MIXED) {
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int e = 4 * (tid + 256 * v);
            const int r = e / M, q = e % M;
#pragma unroll
            for (int i = 0; i < NB; ++i)
                pv[v][i] = *reinterpret_cast<const float4*>(a.P + (((size_t)l * nb + i) * M + r0 + r) * M + q);
        }
    }
    stash();
    if constexpr (MIXED) plane_put<PR, TAIL>(planes_of(fbeg), pl, reinterpret_cast<float2*>(coef));
    // every load so far (the basis pixels included) complete here, once: the loop body's waits then only
    // count what the body itself issued, and a later iteration's epilogue does not wait for the previous
    // iteration's stores on the basis pixels' account (vmcnt(0); expcnt and lgkmcnt at their maxima)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();                                        // spectra and plane coefficients

    // one iteration: NF frames from f0, whose spectra and plane coefficients are in LDS.  PF: the next
    // iteration's are requested after the transforms and put into LDS at the end (waiting for them then
    // passes over this iteration's stores only); FULL: all NF frames lie in the run.  Both are compile-time,
    // so the body has no branches that would blur the counts the compiler's waits are based on.
    auto body = [&](int f0, auto pf, auto full) {
        constexpr bool PF = decltype(pf)::value, FULL = decltype(full)::value;
        // packed C2R: Z[q] = A[q] + i B[q] over the Hermitian extensions of the team's two rows
        float2 x[S::N1];
        {
            const float2* A = reg;
            const float2* B = reg + Kh;
#pragma unroll
            for (int n1 = 0; n1 < S::N1; ++n1) {
                const int q = S::N2 * n1 + t;
                float2 z;
                if (q == M / 2) {
                    z = make_float2(0.f, 0.f);      // Nyquist column: B = 0 there, C is not written
                } else if (q == 0) {
                    z = make_float2(A[q].x, B[q].x);
                } else if (q < M / 2) {
                    const float2 u = A[q], w = B[q];
                    z = make_float2(u.x - w.y, u.y + w.x);
                } else {
                    const float2 u = A[M - q], w = B[M - q];
                    z = make_float2(u.x + w.y, w.x - u.y);
                }
                x[n1] = z;
            }
        }
        team_sync();                        // the team's own region
        fft_pass1_regs<M, +1>(t, reg, twr, x);
        team_sync();                        // the team's own region
        float2 z[S::N1 / S::T][S::N2];
        fft_pass2_load<M>(t, reg, z);
        team_sync();                        // the team's own region
        {
            float* rows = reinterpret_cast<float*>(reg);    // [2][M]
            fft_pass2_regs<M, +1>(t, z, [&](int p, float2 v) {
                rows[p] = v.x;
                rows[M + p] = v.y;
            });
        }
        if constexpr (PF) {
            issue(f0 + NF);
            if constexpr (MIXED) plane_fetch<PR>(planes_of(f0 + NF), pl);
        }
        __syncthreads();                    // rows of every team

        // epilogue: 4-pixel groups, coalesced stores; a group's basis pixels serve every frame of the block
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int e = 4 * (tid + 256 * v);
            const int r = e / M, q = e % M;
#pragma unroll
            for (int fi = 0; fi < NF; ++fi) {
                const int f = f0 + fi;
                const float* src = reinterpret_cast<const float*>(smem + (fi * TPF + r / 2) * RS) + (r & 1) * M + q;
                float4 o = *reinterpret_cast<const float4*>(src);
                if constexpr (MIXED) {
                    const float* cf = coef + fi * nb;
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        const float c = cf[i];
                        o.x = fmaf(c, pv[v][i].x, o.x);
                        o.y = fmaf(c, pv[v][i].y, o.y);
                        o.z = fmaf(c, pv[v][i].z, o.z);
                        o.w = fmaf(c, pv[v][i].w, o.w);
                    }
                    if constexpr (TAIL) {
                        for (int i = NB; i < nb; ++i) {
                            const float c = cf[i];
                            const float4 pw =
                                *reinterpret_cast<const float4*>(a.P + (((size_t)l * nb + i) * M + r0 + r) * M + q);
                            o.x = fmaf(c, pw.x, o.x);
                            o.y = fmaf(c, pw.y, o.y);
                            o.z = fmaf(c, pw.z, o.z);
                            o.w = fmaf(c, pw.w, o.w);
                        }
                    }
                }
                if (FULL || f < fend) {
                    if constexpr (INTEG) {          // integrator of the closed loop (Alg. 3)
                        const size_t oi = (((size_t)f * L + l) * M + r0 + r) * M + q;
                        const float4 pr = *reinterpret_cast<const float4*>(a.prev + oi);
                        const float keep = 1.f - a.gain;
                        o.x = fmaf(a.gain, o.x, keep * pr.x);
                        o.y = fmaf(a.gain, o.y, keep * pr.y);
                        o.z = fmaf(a.gain, o.z, keep * pr.z);
                        o.w = fmaf(a.gain, o.w, keep * pr.w);
                    }
                    // the layers are not read again by the step: streamed past the caches that hold C and the
                    // basis (non-temporal), at device scope (SC1, measured 0.8 us faster per 64 MORFEO-like frames
                    // than the non-temporal hint alone); one descriptor per (frame, layer) plane of M^2 floats
                    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                    const u32x4 ov = {__float_as_uint(o.x), __float_as_uint(o.y), __float_as_uint(o.z),
                                      __float_as_uint(o.w)};
                    const __amdgpu_buffer_rsrc_t plane = __builtin_amdgcn_make_buffer_rsrc(
                        a.out + ((size_t)f * L + l) * M * M, (short)0, M * M * 4, 0x00020000);
                    __builtin_amdgcn_raw_buffer_store_b128(ov, plane, ((r0 + r) * M + q) * 4, 0, kStoreLayers);
                }
            }
        }
        if constexpr (PF) {
            __syncthreads();                // every epilogue done with the regions and the coefficients
            stash();
            if constexpr (MIXED) plane_put<PR, TAIL>(planes_of(f0 + NF), pl, reinterpret_cast<float2*>(coef));
            __syncthreads();
        }
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    int f0 = fbeg;
    for (; f0 + NF < fend; f0 += NF) body(f0, yes{}, yes{});
    if (f0 + NF == fend) body(f0, no{}, yes{});
    else body(f0, no{}, no{});
}

bool out_rows_supported(int M, int RT) {
    if (RT != 8 && RT != 16 && RT != 32) return false;
    if (RT > M || RT * M < 1024) return false;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    return RT / 2 <= 256 / T;
}

int out_frames_per_iter(int M, int RT) {
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    return (256 / T) / (RT / 2);
}

size_t out_lds_bytes(int M, int RT, int nb) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const int T = M == 256 ? 16 : (M == 32 ? 4 : 8);
    const int NF = out_frames_per_iter(M, RT);
    return (size_t)(256 / T) * (N1 * (N2 + 1) + 2) * sizeof(float2) + (size_t)NF * nb * sizeof(float);
}

namespace {

template <int M, int RT, int NB, bool INTEG>
hipError_t launch_out_k(const OutArgs& a, int frames, hipStream_t s) {
    const size_t lds = out_lds_bytes(M, RT, a.nb);
    allow_large_lds(reinterpret_cast<const void*>(&out_kernel<M, RT, NB, INTEG>));
    const int fpb = a.frames_per_block;
    const int nwork = (M / RT) * a.L * ((frames + fpb - 1) / fpb);
    hipLaunchKernelGGL((out_kernel<M, RT, NB, INTEG>), dim3((nwork + 7) / 8 * 8), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int M, int RT, int NB>
hipError_t launch_out_t(const OutArgs& a, int frames, hipStream_t s) {
    return a.prev ? launch_out_k<M, RT, NB, true>(a, frames, s) : launch_out_k<M, RT, NB, false>(a, frames, s);
}

template <int M, int NB>
hipError_t launch_out_rt(const OutArgs& a, int rt, int frames, hipStream_t s) {
    if constexpr (M >= 128) {
        if (rt == 8) return launch_out_t<M, 8, NB>(a, frames, s);
    }
    if constexpr (M >= 64) {
        if (rt == 16) return launch_out_t<M, 16, NB>(a, frames, s);
    }
    if (rt == 32) return launch_out_t<M, 32, NB>(a, frames, s);
    return hipErrorInvalidValue;
}

// basis images in registers: exactly 2, 4 or 6 of them (one to three natural stars), else the first 8 (and
// the rest re-read per frame)
template <int M>
hipError_t launch_out_m(const OutArgs& a, int rt, int frames, hipStream_t s) {
    switch (a.nb) {
        case 0: return launch_out_rt<M, 0>(a, rt, frames, s);
        case 2: return launch_out_rt<M, 2>(a, rt, frames, s);
        case 4: return launch_out_rt<M, 4>(a, rt, frames, s);
        case 6: return launch_out_rt<M, 6>(a, rt, frames, s);
        default: return launch_out_rt<M, 8>(a, rt, frames, s);
    }
}

}  // namespace

hipError_t launch_out(int M, const OutArgs& a, int rows_per_block, int frames, hipStream_t s) {
    if (!out_rows_supported(M, rows_per_block) || a.frames_per_block < 1) return hipErrorInvalidValue;
    switch (M) {
        case 32: return launch_out_m<32>(a, rows_per_block, frames, s);
        case 64: return launch_out_m<64>(a, rows_per_block, frames, s);
        case 128: return launch_out_m<128>(a, rows_per_block, frames, s);
        case 256: return launch_out_m<256>(a, rows_per_block, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace safr
