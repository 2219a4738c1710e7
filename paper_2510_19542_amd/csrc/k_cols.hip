// Column pass of SAFR's hard-real-time step (Alg. 1), fused:
//   1. column FFT (length M) of each star's row spectrum R[.][k][.] (the input
//      is nonzero in the n pupil rows only, read directly from the row pass);
//   2. per-frequency apply b_l(j, k) = sum_g B[k][l][g][j] d_g(j, k) with the
//      group's FP32 B (Eq. sparseM: B is diagonal in frequency);
//   3. inverse column FFT of each layer spectrum, written to C in row tiles of 8
//      (C[f][l][p / 8][k][p % 8]).
// Split tomography (Sec. 3.3): for the laser stars of a mixed asterism the
// least-squares plane b x + c y over the pupil (from the row-pass moments) is
// removed; the transform being linear, that is d_g -= b DFT2(x mask) +
// c DFT2(y mask), with the two transforms precomputed in FP64 per plan.  The
// natural stars are added in the output pass.
//
// Only the columns k < M/2 are processed: B vanishes on the Nyquist column, whose
// layer spectra the output pass takes as zero.
//
// One block of 256 threads owns CPW = 256 / M columns and a run of frames,
// transformed NF frames at a time.  LDS holds one slot of team_lds<M>() float2
// per (column, frame, star-or-layer); a slot is in turn a transform's exchange
// buffer and its spectrum: forward transforms leave d_g in the star slots, the
// apply (thread = column, frequency j) reads every d_g(j) of its frames into
// registers and writes b_l(j) into the layer slots (which overlap the star
// slots only at its own index j), and the inverse transforms run in place in
// the layer slots.  Phases that overwrite a slot first take what they need into
// registers, with a barrier in between.  The forward inputs
// of an iteration are all requested before its first transform.
//
// B is stored per block of columns as [l][g][column][j] (thread t owns entries
// t, t + 256, ...) and is read from global memory at each apply, once for NF
// frames.  Blocks are mapped XCD-aware: the blocks of one column block (all
// its frame runs) are consecutive on the same XCD, so its B stays in that
// XCD's L2.
//
// cols_kernel<M, NF, G, L, MODE> with compile-time G, L (the configured
// geometries) keeps d in registers; G = L = 0 is the generic kernel (any shape,
// NF = 1, separate star and layer slots, d re-read from LDS).  The apply reads
// the G entries of B of each layer just before its products: requesting all
// L x G entries up front (or keeping them in registers across frames) does not
// fit the register file next to the transforms at M = 256 and spills.
#include "fft_device.h"
#include "safr_internal.h"

namespace safr {

namespace {

// d - (b X + c Y) with (b, c) = cf: two FMAs per part
__device__ __forceinline__ float2 remove_plane(float2 d, float2 cf, float2 xh, float2 yh) {
    return make_float2(fmaf(-cf.y, yh.x, fmaf(-cf.x, xh.x, d.x)), fmaf(-cf.y, yh.y, fmaf(-cf.x, xh.y, d.y)));
}

// acc + b d as four FMAs (written as one expression, the product difference would be formed first and
// cost a multiply, an FMA and an add per part)
__device__ __forceinline__ float2 cmac(float2 acc, float2 b, float2 d) {
    acc.x = fmaf(b.x, d.x, acc.x);
    acc.x = fmaf(-b.y, d.y, acc.x);
    acc.y = fmaf(b.x, d.y, acc.y);
    acc.y = fmaf(b.y, d.x, acc.y);
    return acc;
}

// Raw buffer access to the block's B slice: the descriptor is uniform (scalar registers) and each
// (l, g) entry is one 32-bit lane offset plus a scalar offset, so the loop-invariant addresses of the
// L x G loads do not each occupy a 64-bit vector register pair.  Word 3 is the gfx9-family default.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float2 load_b(__amdgpu_buffer_rsrc_t r, int lane_bytes, int entry) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, lane_bytes, entry * 2048, 0));
}

__device__ __forceinline__ float2 load_f2(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

// Stores of the layer spectra C carry device scope (cache policy SC1): measured, they leave more of the
// block's B resident in L2 between the frame groups (the column pass 2.4 us faster per 64 MORFEO-like
// frames; the non-temporal hint instead slows it, and the output pass that reads C, down).
constexpr int kStoreC = 16;

__device__ __forceinline__ void store_f2(__amdgpu_buffer_rsrc_t r, int byte_off, float2 v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, byte_off, 0, kStoreC);
}

// byte offset beyond every descriptor's range: a buffer store there is dropped by the hardware (lanes without
// work store there instead of branching around the store)
constexpr int kDropOffset = 0x7FFFFFF8;

// linear block -> (column block, frame run), XCD-contiguous (blocks are dealt to the 8 XCDs round-robin)
__device__ __forceinline__ bool xcd_work(int nwork, int& w) {
    const int b = blockIdx.x, per = gridDim.x / 8;
    w = (b % 8) * per + b / 8;
    return w < nwork;
}

}  // namespace

template <int M, int NF, int GC, int LC, int MODE, int LSPLIT = 1, int NN = 0, bool MF = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M >= 128 ? 2 : 3))) void cols_kernel(ColArgs a) {
    static_assert(!MF || (GC > 0 && NF == 4 && LSPLIT == 1), "the matrix-core apply takes 4 frames as its rows");
    using S = FftShape<M>;
    constexpr int T = S::T, N1 = S::N1, NTEAM = 256 / T, TL = team_lds<M>() + 2;   // slot stride, 4 banks apart
    constexpr int CPW = 256 / M, Kh = M / 2 + 1;
    constexpr bool FIX = GC > 0;
    const int G = FIX ? GC : a.grp.G;
    const int L = FIX ? LC : a.L;
    // slots: star slots [c][f][g] at 0, layer slots [c][f][l] at LS (overlapping when FIX)
    const int SPF = FIX ? (GC > LC ? GC : LC) : G + L;          // slots per (column, frame)
    const int LS = FIX ? 0 : G;

    extern __shared__ float2 smem[];
    float2* slots = smem;                                      // [CPW][NF][SPF][TL]
    // the matrix-core apply reads and writes one slot of each of the 4 frames per instruction: frames are
    // padded to 8 float2 past a multiple of 32 apart, so the 4 frames' 8-pair runs of a half wavefront fall
    // in distinct banks
    constexpr int FPAD = MF ? (8 - ((GC > LC ? GC : LC) * TL) % 32 + 32) % 32 : 0;
    const int FSTR = SPF * TL + FPAD;                           // float2 per (column, frame)
    float2* coef = slots + (size_t)CPW * NF * FSTR;            // [NF][G]

    // columns k < M/2 only: B vanishes on the Nyquist column k = M/2, so its layer spectra are zero and
    // the output pass takes them as such without reading C there
    constexpr int KC = M / 2;
    const int kblocks = KC / CPW;
    const int runs = (a.frames + a.frames_per_block - 1) / a.frames_per_block;
    int w;
    if (!xcd_work(kblocks * runs * LSPLIT, w)) return;         // the whole block leaves before any barrier
    // layer split (launches with fewer blocks than CUs): the LSPLIT blocks of a column each transform all
    // stars and apply and invert LB of the layers, starting at l0
    constexpr int LB = FIX ? (LC + LSPLIT - 1) / LSPLIT : 1;
    const int ls = w % LSPLIT;
    w /= LSPLIT;
    const int l0 = ls * LB;
    const int nl = FIX ? min(LB, LC - l0) : L;                 // layers of this block
    const int kb = w / runs, run = w - kb * runs;
    const int fbeg = run * a.frames_per_block;
    const int fend = min(a.frames, fbeg + a.frames_per_block);
    const int tid = threadIdx.x, team = tid / T, t = tid % T;
    const int c = tid / M, j = tid % M;                        // apply: column in block, frequency
    const int k = kb * CPW + c;                                // < KC: blocks past the work left above
    auto slot = [&](int cc, int f, int s) { return slots + (size_t)(cc * NF + f) * FSTR + (size_t)s * TL; };

    // forward tasks: (column, frame, star); rounds of NTEAM teams
    const int ftasks = CPW * NF * G;
    constexpr int FR_MAX = FIX ? (CPW * NF * GC + NTEAM - 1) / NTEAM : 1;
    constexpr int FR_UNROLL = FR_MAX;                          // run-time round counts are not unrolled
    float2 xf[FR_MAX][N1];
    // Deferred inverse tail (compile-time shapes with more layers than stars, one column per block): the
    // inverse transforms run layers l < G first and l >= G last, and the tasks of the last inverse round
    // (all with l >= G, slots no forward transform writes) run in the teams the next frame group's last
    // forward round leaves idle, whole wavefronts of them, so each group takes one round less.
    constexpr int IT_FIX = CPW * NF * LB, IR_FIX = FIX ? (IT_FIX + NTEAM - 1) / NTEAM : 1;
    constexpr int F_LAST = CPW * NF * GC - (FR_MAX - 1) * NTEAM;        // forward tasks of the last round
    constexpr int I_LAST = IT_FIX - (IR_FIX - 1) * NTEAM;               // inverse tasks of the last round
    constexpr int TPWV = 64 / T;                                        // teams per wavefront
    constexpr bool DEFER = FIX && LSPLIT == 1 && CPW == 1 && LC > GC && IR_FIX > 1 && I_LAST > 0 &&
                           I_LAST <= NF * (LC - GC) && F_LAST % TPWV == 0 && F_LAST + I_LAST <= NTEAM;
    constexpr int IR_UNROLL = IR_FIX;
    // R of frames f0 .. f0 + NF - 1 through one descriptor (byte offsets stay below 2^31)
    const int fstride = a.J * Kh * a.n;                        // float2 per frame of R
    // pupil rows: compile-time when NN > 0.  Team thread t's inputs are the column's rows N2 n1 + t, so only
    // the n1 in [WLO, WHI] can meet the pupil rows p0 .. p0 + n - 1; the others are literal zeros (no load,
    // no register)
    constexpr int P0 = NN > 0 ? (M - NN + 1) / 2 : 0;
    constexpr int WLO = NN > 0 && P0 - T + 1 > 0 ? (P0 - T + 1 + S::N2 - 1) / S::N2 : 0;
    constexpr int WHI = NN > 0 ? ((P0 + NN - 1) / S::N2 < N1 - 1 ? (P0 + NN - 1) / S::N2 : N1 - 1) : N1 - 1;
    const int pn = NN > 0 ? NN : a.n, pp0 = NN > 0 ? P0 : a.p0;
    // every load is issued (rows outside the pupil, idle teams and frames past the run read offset 0 of the
    // descriptor and are replaced by zero), so the loads need no branches and their waits can be counted
    auto load_fwd = [&](int f0, int round, float2 (&x)[N1]) {
        const int task = round * NTEAM + team;
        const int cc = task / (NF * G), rem = task - cc * (NF * G);
        const int fl = rem / G, g = rem - fl * G;
        const int kk = kb * CPW + cc, f = f0 + fl;
        const bool ok = task < ftasks && kk < KC && f < fend;
        const int nfr = min(NF, fend - f0);
        const __amdgpu_buffer_rsrc_t rr = block_rsrc(a.R + (size_t)f0 * fstride, (unsigned)(nfr * fstride * 8));
        const int colb = ((fl * a.J + g) * Kh + kk) * a.n;       // R holds the group's stars first
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            if (n1 < WLO || n1 > WHI) {
                x[n1] = make_float2(0.f, 0.f);
                continue;
            }
            const int pr = S::N2 * n1 + t - pp0;
            const bool in = ok && pr >= 0 && pr < pn;
            const float2 v = load_f2(rr, in ? (colb + pr) * 8 : 0);
            x[n1] = in ? v : make_float2(0.f, 0.f);
        }
    };

    float2 twr[N1];                                            // this thread's pass-1 twiddles
    load_pass1_twiddles<M>(a.tw, t, twr);
    float2 xh = make_float2(0.f, 0.f), yh = make_float2(0.f, 0.f);
    if (MODE != 0) {
        xh = a.Xh[(size_t)k * M + j];
        yh = a.Yh[(size_t)k * M + j];
    }
    const __amdgpu_buffer_rsrc_t Brs = block_rsrc(a.B + (size_t)kb * L * G * 256, (unsigned)(L * G * 256 * 8));

    // Software pipelined over the block's frames: the loop body runs the inverse transforms of one iteration
    // (NF frames) and then the forward transforms and the apply of the next.  With the pupil size at compile
    // time (PFN: only the inputs that can meet the pupil rows are held) the next iteration's first forward
    // inputs are requested at the start of the body, before its layer-spectrum stores: the vector-memory
    // counter counts loads and stores in issue order, so inputs requested after those stores could only be
    // waited for together with them, and inputs carried over the loop's back edge would be waited for when
    // the compiler copies them into place.  Otherwise (all M inputs of a round in registers) they are
    // requested at the start of the forward transforms.  Each later round's inputs are requested after the
    // previous round's first pass, so at most two rounds of inputs are held at once.
    //
    // forward transforms and apply of the NF frames from f0 (for compile-time shapes their first round's
    // inputs are in xf[0] already)
    // The apply on the matrix cores (MF: compile-time shapes with NF = 4).  v_mfma_f32_4x4x1f32 computes 16
    // independent 4 x 4 outer products per wavefront: block = (column, frequency) pair, rows = the 4 frames,
    // columns = 4 layers, accumulated over the stars.  Lane 4b + m holds row m of block b's A operand and
    // column m of its B operand; the result for (row m, column n) lands in lane 4b + n, register m.  The
    // complex product is four real ones: Re b += Re d Re B - Im d Im B, Im b += Im d Re B + Re d Im B.  Each
    // wavefront takes 4 groups of 16 pairs (its 64 pairs): it reads the d of all frames and stars of a group
    // into registers, then writes the group's b into the layer slots (in place: only its own pairs).
    // B streamed in steps s = (group q, star g) of MLBK float2 per lane (its layer blocks), MPF steps ahead
    constexpr int MLBK = MF ? (LC + 3) / 4 : 1;                // layer blocks of 4 (padded with zero B)
    // (MPF + 1 divides the steps of a group, so the buffer of each step is known at compile time with the
    // group loop kept rolled)
    constexpr int MPF = (MF ? GC : 1) % 3 == 0 ? 2 : 1, MSTEPS = 4 * (MF ? GC : 1);
    [[maybe_unused]] float2 mb[MPF + 1][MLBK];
    [[maybe_unused]] float2 mxy[2][2];                         // Xh, Yh of the lane's pair for groups q, q + 1
    [[maybe_unused]] auto mfma_bload = [&](int step, float2 (&dst)[MLBK]) {
        if constexpr (MF) {
            const int q = step / GC, g = step % GC;
            const int wave = tid >> 6, lane = tid & 63;
            const __amdgpu_buffer_rsrc_t bmr =
                block_rsrc(a.Bm + (size_t)kb * 16 * MLBK * GC * 64, (unsigned)(16 * MLBK * GC * 64 * 8));
#pragma unroll
            for (int lb = 0; lb < MLBK; ++lb)
                dst[lb] = load_f2(bmr, ((((wave * 4 + q) * GC + g) * MLBK + lb) * 64 + lane) * 8);
        }
    };
    [[maybe_unused]] auto mfma_xyload = [&](int q, float2 (&dst)[2]) {
        if constexpr (MF && MODE != 0) {
            const int pr = (((tid >> 6) * 4 + q) * 16 + ((tid & 63) >> 2));
            dst[0] = a.Xh[(size_t)(kb * CPW + pr / M) * M + pr % M];
            dst[1] = a.Yh[(size_t)(kb * CPW + pr / M) * M + pr % M];
        }
    };
    // requested before the barrier that precedes the apply: the first MPF steps of B and group 0's Xh, Yh
    [[maybe_unused]] auto mfma_prefetch = [&]() {
        if constexpr (MF) {
#pragma unroll
            for (int sp = 0; sp < MPF; ++sp) mfma_bload(sp, mb[sp]);
            mfma_xyload(0, mxy[0]);
        }
    };
    // The apply on the matrix cores (v_mfma_f32_4x4x1_16b_f32: 16 independent 4 x 4 blocks per wavefront,
    // K = 1).  Block b of a wavefront takes one (column, frequency) pair: rows = 4 layers, columns = the
    // NF = 4 frames, accumulated over the stars.  Lane 4b + m holds row m of block b's A operand (B of layer
    // m) and column m of its B operand (d of frame m); the result for (row m, column n) lands in lane 4b + n,
    // register m, so each lane reads and writes its own frame.  The complex product is four real ones:
    // Re b += Re B Re d - Im B Im d, Im b += Re B Im d + Im B Re d.  Each
    // wavefront takes 4 groups of 16 pairs (its 64 pairs): it reads the d of all frames and stars of a group
    // into registers, then writes the group's b into the layer slots (in place: only its own pairs).  For
    // each star the 2 MLBK accumulators (real and imaginary part of each layer block) are independent chains.
    [[maybe_unused]] auto apply_mfma = [&](int f0) {
        if constexpr (MF) {
            typedef float f32x4 __attribute__((ext_vector_type(4)));
            const int wave = tid >> 6, lane = tid & 63, m4 = lane & 3;
            (void)f0;
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                const int pr = (wave * 4 + q) * 16 + (lane >> 2); // (column, frequency) pair of the lane's block
                const int cq = pr / M, jq = pr % M;
                float ar[GC], ai[GC];
#pragma unroll
                for (int g = 0; g < GC; ++g) {
                    float2 d = slot(cq, m4, g)[jq];             // frame m4 of the lane's pair
                    if constexpr (MODE != 0) d = remove_plane(d, coef[m4 * GC + g], mxy[0][0], mxy[0][1]);
                    ar[g] = d.x;
                    ai[g] = d.y;
                }
                mfma_xyload(min(q + 1, 3), mxy[1]);
                f32x4 accR[MLBK], accI[MLBK];
#pragma unroll
                for (int lb = 0; lb < MLBK; ++lb) {
                    accR[lb] = (f32x4){0.f, 0.f, 0.f, 0.f};
                    accI[lb] = (f32x4){0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int g = 0; g < GC; ++g) {
                    const int step = q * GC + g;
                    // clamped on the last group (a repeated load, never used): no branch around it
                    mfma_bload(min(step + MPF, MSTEPS - 1), mb[(g + MPF) % (MPF + 1)]);
                    const float2* bv = mb[g % (MPF + 1)];
#pragma unroll
                    for (int lb = 0; lb < MLBK; ++lb) {
                        accR[lb] = __builtin_amdgcn_mfma_f32_4x4x1f32(bv[lb].x, ar[g], accR[lb], 0, 0, 0);
                        accI[lb] = __builtin_amdgcn_mfma_f32_4x4x1f32(bv[lb].x, ai[g], accI[lb], 0, 0, 0);
                    }
#pragma unroll
                    for (int lb = 0; lb < MLBK; ++lb) {
                        accR[lb] = __builtin_amdgcn_mfma_f32_4x4x1f32(bv[lb].y, -ai[g], accR[lb], 0, 0, 0);
                        accI[lb] = __builtin_amdgcn_mfma_f32_4x4x1f32(bv[lb].y, ar[g], accI[lb], 0, 0, 0);
                    }
                }
                // lane 4b + f holds frame f of layers 4 lb .. 4 lb + 3 (register r = layer 4 lb + r)
#pragma unroll
                for (int lb = 0; lb < MLBK; ++lb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (lb * 4 + r < LC) slot(cq, m4, lb * 4 + r)[jq] = make_float2(accR[lb][r], accI[lb][r]);
                mxy[0][0] = mxy[1][0];
                mxy[0][1] = mxy[1][1];
            }
        }
    };
    // inverse transforms of the NF frames from f0 (the apply's layer spectra complete in LDS)
    // 3. inverse column transforms of the layer slots, in place, written to C.  Compile-time shapes run a
    // fixed number of rounds with every lane storing: a lane without a task (or whose frame lies past the
    // run) stores to an offset beyond the descriptor's range, which the hardware drops, so the stores need
    // no branches and the waits after them can be counted.
    const int itasks = CPW * NF * nl;
    const size_t cfr = (size_t)L * Kh * M;                     // float2 per frame of C
    auto c_rsrc = [&](int f0) __attribute__((always_inline)) {
        return block_rsrc(a.C + c_index(f0, 0, L, M, 0, 0), (unsigned)(min(NF, fend - f0) * cfr * 8));
    };
    auto inv_task = [&](int f0, int task, __amdgpu_buffer_rsrc_t cr) __attribute__((always_inline)) {
        int cc, fl, l;
        if constexpr (DEFER) {                                  // layers below G first, the others last
            cc = 0;
            if (task < NF * GC) {
                fl = task / GC;
                l = task - fl * GC;
            } else {
                const int t2 = task - NF * GC;
                fl = t2 / (LC - GC);
                l = GC + t2 - fl * (LC - GC);
            }
        } else {
            cc = task / (NF * nl);
            const int rem = task - cc * (NF * nl);
            fl = rem / nl;
            l = rem - fl * nl;
        }
        const int kk = kb * CPW + cc, f = f0 + fl;
        const bool active = task < itasks;
        float2* sl = active ? slot(cc, fl, LS + l) : slots;
        float2 x[N1];
        if (active) {
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) x[n1] = sl[S::N2 * n1 + t];
        }
        team_sync();                            // the team's own slot
        if (active) fft_pass1_regs<M, +1>(t, sl, twr, x);   // idle teams must not write another team's slot
        team_sync();                            // the team's own slot
        // idle teams read slot 0 (another team's data, possibly mid-transform) and drop their stores
        const bool store = active && f < fend;
        const int base = store ? (int)(c_index(fl, l0 + l, L, M, kk, 0)) : 0;
        fft_pass2<M, +1>(t, sl, [&](int p, float2 v) {
            store_f2(cr, store ? (base + (p >> 3) * (Kh * 8) + (p & 7)) * 8 : kDropOffset, v);
        });
    };
    constexpr bool PFN = FIX && NN > 0;        // next inputs requested ahead of the stores (pupil size known)
    // fprev: the previous frame group, whose deferred inverse tail runs in the last forward round (with tail;
    // both calls are inlined with a constant tail)
    auto fwd_apply = [&](int f0, int fprev, bool tail) __attribute__((always_inline)) {
        const bool TAIL = DEFER && tail;
        const __amdgpu_buffer_rsrc_t crp = c_rsrc(tail ? fprev : f0);
        if constexpr (FIX && !PFN) load_fwd(f0, 0, xf[0]);
        // tip/tilt plane coefficients of this iteration's frames, requested now and stored after the
        // forward transforms
        const PlaneArgs pa{a.planes, a.plane_nch, a.J, G, f0, fend, min(NF, fend - f0) * G, 0};
        float2 pl[1];
        if (MODE != 0) plane_fetch<1>(pa, pl);
        __syncthreads();                                        // previous inverse transforms done with the slots
        // 1. forward column transforms into the star slots
        const int frounds = FIX ? FR_MAX : (ftasks + NTEAM - 1) / NTEAM;
#pragma unroll FR_UNROLL
        for (int r = 0; r < frounds; ++r) {
            if (TAIL && r == FR_MAX - 1 && team >= F_LAST) {    // whole wavefronts: a scalar branch
                if (team < F_LAST + I_LAST) inv_task(fprev, (IR_FIX - 1) * NTEAM + team - F_LAST, crp);
                continue;
            }
            const int task = r * NTEAM + team;
            const int cc = task / (NF * G), rem = task - cc * (NF * G);
            const int fl = rem / G, g = rem - fl * G;
            const bool active = task < ftasks;
            float2* sl = active ? slot(cc, fl, g) : slots;
            float2 x[N1];
            if constexpr (FIX) {
#pragma unroll
                for (int n1 = 0; n1 < N1; ++n1) x[n1] = xf[r][n1];
            } else {
                load_fwd(f0, r, x);
            }
            if (active) fft_pass1_regs<M, -1>(t, sl, twr, x);
            if constexpr (FIX) {
                if (r + 1 < FR_MAX) load_fwd(f0, r + 1, xf[r + 1 < FR_MAX ? r + 1 : r]);
            }
            team_sync();                        // the team's own slot
            float2 z[N1 / T][S::N2];
            if (active) fft_pass2_load<M>(t, sl, z);
            team_sync();                        // the team's own slot
            if (active) fft_pass2_regs<M, -1>(t, z, [&](int jj, float2 v) { sl[jj] = v; });
        }
        // B of the block's first layers, requested before the barrier; later layers BD - 1 ahead of use: one
        // when four frames share each B (a deeper prefetch holds more registers and measured slower), two for
        // fewer frames (one-frame calls wait on B sooner)
        constexpr int BD = NF >= 4 ? 2 : 3;                     // B buffers in flight
        float2 bq[BD][FIX ? GC : 1];
        if constexpr (MF) mfma_prefetch();
        if constexpr (FIX && !MF) {
#pragma unroll
            for (int q = 0; q < BD - 1; ++q) {
                if (q < LB && (LSPLIT == 1 || q < nl)) {
#pragma unroll
                    for (int g = 0; g < GC; ++g) bq[q][g] = load_b(Brs, tid * 8, (l0 + q) * GC + g);
                }
            }
        }
        // tip/tilt plane coefficients of this iteration's frames (used by the apply, after the barrier)
        static_assert(NF * (FIX ? GC : kMaxG) <= 256 / kPlaneLanes, "one round of plane lanes takes every pair");
        if (MODE != 0) plane_put<1, false>(pa, pl, coef);
        __syncthreads();

        // 2. apply: b_l(j) = sum_g B[l][g][j] d_g(j) for the NF frames
        if constexpr (MF) {
            apply_mfma(f0);
        } else if constexpr (FIX) {
            float2 dv[NF][GC];
#pragma unroll
            for (int fl = 0; fl < NF; ++fl)
#pragma unroll
                for (int g = 0; g < GC; ++g) {
                    const float2 d = slot(c, fl, g)[j];
                    dv[fl][g] = MODE != 0 ? remove_plane(d, coef[fl * GC + g], xh, yh) : d;
                }
            // B of layer l + BD - 1 is requested before the products of layer l
#pragma unroll
            for (int l = 0; l < LB; ++l) {
                if (LSPLIT > 1 && l >= nl) break;
                const float2* bv = bq[l % BD];
                if (l + BD - 1 < LB && (LSPLIT == 1 || l + BD - 1 < nl)) {
#pragma unroll
                    for (int g = 0; g < GC; ++g) bq[(l + BD - 1) % BD][g] = load_b(Brs, tid * 8, (l0 + l + BD - 1) * GC + g);
                }
#pragma unroll
                for (int fl = 0; fl < NF; ++fl) {
                    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                    for (int g = 0; g < GC; ++g) acc = cmac(acc, bv[g], dv[fl][g]);
                    slot(c, fl, l)[j] = acc;
                }
            }
        } else {
            for (int l = 0; l < L; ++l) {
                float2 acc = make_float2(0.f, 0.f);
                for (int g = 0; g < G; ++g) {
                    float2 d = slot(c, 0, g)[j];
                    if (MODE != 0) d = remove_plane(d, coef[g], xh, yh);
                    const float2 bv = load_b(Brs, tid * 8, l * G + g);
                    acc = cmac(acc, bv, d);
                }
                slot(c, 0, LS + l)[j] = acc;
            }
        }
    };
    // all rounds, or (the deferred tail) all but the last
    auto inverse = [&](int f0, bool all) __attribute__((always_inline)) {
        const int irounds = FIX ? (DEFER && !all ? IR_FIX - 1 : IR_FIX) : (itasks + NTEAM - 1) / NTEAM;
        const __amdgpu_buffer_rsrc_t cr = c_rsrc(f0);
#pragma unroll IR_UNROLL
        for (int r = 0; r < irounds; ++r) inv_task(f0, r * NTEAM + team, cr);
    };
    if constexpr (PFN) load_fwd(fbeg, 0, xf[0]);
    fwd_apply(fbeg, 0, false);
    int f0 = fbeg;
    for (; f0 + NF < fend; f0 += NF) {
        __syncthreads();                                        // the apply's layer spectra
        if constexpr (PFN) load_fwd(f0 + NF, 0, xf[0]);         // ahead of this iteration's stores
        inverse(f0, false);
        fwd_apply(f0 + NF, f0, true);                           // with this group's deferred inverse tail
    }
    __syncthreads();
    inverse(f0, true);
}

// B in the matrix-core lane layout (see ColArgs::Bm): one thread per output float2
__global__ void pack_mfma_b_kernel(int M, int L, int G, const float2* __restrict__ B32, float2* __restrict__ Bm,
                                   size_t count) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int LBK = (L + 3) / 4;
    const int lane = (int)(e % 64);
    size_t r = e / 64;
    const int lb = (int)(r % LBK);
    r /= LBK;
    const int g = (int)(r % G);
    r /= G;
    const int grp = (int)(r % 16);
    const size_t kb = r / 16;
    const int l = lb * 4 + lane % 4, pr = grp * 16 + lane / 4;
    Bm[e] = l < L ? B32[((kb * L + l) * G + g) * 256 + pr] : make_float2(0.f, 0.f);
}

size_t mfma_b_count(int M, int L, int G) {
    const int kblocks = (M / 2) / (256 / M);                  // the columns k < M/2 of the column pass
    return (size_t)kblocks * 16 * ((L + 3) / 4) * G * 64;
}

hipError_t launch_pack_mfma_b(int M, int L, int G, const float2* B32, float2* Bm, hipStream_t s) {
    const size_t count = mfma_b_count(M, L, G);
    hipLaunchKernelGGL(pack_mfma_b_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, M, L, G, B32, Bm,
                       count);
    return hipGetLastError();
}

size_t cols_lds_bytes(int M, int G, int L, int nf, bool fixed, bool mf) {
    const int N1 = M == 32 ? 8 : (M == 64 ? 8 : 16), N2 = M / N1;
    const size_t tl = (size_t)N1 * (N2 + 1) + 2;
    const int spf = fixed ? (G > L ? G : L) : G + L;
    const size_t fpad = mf ? (size_t)((8 - (int)((spf * tl) % 32) + 32) % 32) : 0;
    return ((size_t)(256 / M) * nf * (spf * tl + fpad) + (size_t)nf * G) * sizeof(float2);
}

namespace {

template <class K>
hipError_t launch_cols_kernel(K kernel, int M, int nf, bool fixed, const ColArgs& a, int frames, hipStream_t s,
                              int lsplit = 1, bool mf = false) {
    const int CPW = 256 / M;
    const size_t lds = cols_lds_bytes(M, a.grp.G, a.L, nf, fixed, mf);
    const int kblocks = (M / 2) / CPW;                       // the Nyquist column is not transformed
    const int runs = (frames + a.frames_per_block - 1) / a.frames_per_block;
    const int nblk = (kblocks * runs * lsplit + 7) / 8 * 8;
    allow_large_lds(reinterpret_cast<const void*>(kernel));
    hipLaunchKernelGGL(kernel, dim3(nblk), dim3(256), lds, s, a);
    return hipGetLastError();
}

// shapes with a compile-time kernel: (M, L, group size, mode, pupil size of the configured workload); a
// matching shape with another pupil size takes the same kernels with the pupil size at run time
#define SAFR_FIXED_SHAPES(X) \
    X(256, 9, 6, 1, 69)      \
    X(256, 9, 6, 0, 69)      \
    X(128, 5, 6, 0, 41)      \
    X(64, 2, 4, 0, 33)       \
    X(64, 3, 4, 0, 33)

// fewer column blocks than CUs (one-frame calls at M = 256): split the layers of each column over two blocks
constexpr int kCUs = 256;

template <int M, int G, int L, int MODE, int NN>
hipError_t launch_fixed_n(const ColArgs& a, int nf, int frames, hipStream_t s) {
    const int CPW = 256 / M, kblocks = (M / 2) / CPW;
    const int runs = (frames + a.frames_per_block - 1) / a.frames_per_block;
    if (nf == 1 && L >= 2 && kblocks * runs * 2 <= kCUs + kCUs / 8)
        return launch_cols_kernel(&cols_kernel<M, 1, G, L, MODE, 2, NN>, M, 1, true, a, frames, s, 2);
    switch (nf) {
        case 1: return launch_cols_kernel(&cols_kernel<M, 1, G, L, MODE, 1, NN>, M, 1, true, a, frames, s);
        case 2: return launch_cols_kernel(&cols_kernel<M, 2, G, L, MODE, 1, NN>, M, 2, true, a, frames, s);
        case 4:
            return a.Bm ? launch_cols_kernel(&cols_kernel<M, 4, G, L, MODE, 1, NN, true>, M, 4, true, a, frames, s, 1,
                                             true)
                        : launch_cols_kernel(&cols_kernel<M, 4, G, L, MODE, 1, NN>, M, 4, true, a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

template <int M, int G, int L, int MODE, int NN>
hipError_t launch_fixed(const ColArgs& a, int nf, int frames, hipStream_t s) {
    return a.n == NN ? launch_fixed_n<M, G, L, MODE, NN>(a, nf, frames, s)
                     : launch_fixed_n<M, G, L, MODE, 0>(a, nf, frames, s);
}

template <int M>
hipError_t launch_generic(const ColArgs& a, int frames, hipStream_t s) {
    return a.grp.mode ? launch_cols_kernel(&cols_kernel<M, 1, 0, 0, 1>, M, 1, false, a, frames, s)
                      : launch_cols_kernel(&cols_kernel<M, 1, 0, 0, 0>, M, 1, false, a, frames, s);
}

}  // namespace

bool cols_fixed_shape(int M, int L, int G, int mode) {
#define SAFR_MATCH(m, l, g, md, nn) \
    if (M == m && L == l && G == g && mode == md) return true;
    SAFR_FIXED_SHAPES(SAFR_MATCH)
#undef SAFR_MATCH
    return false;
}

hipError_t launch_cols(int M, const ColArgs& a, int nf, int frames, hipStream_t s) {
    const int G = a.grp.G, mode = a.grp.mode;
    if (a.prefetch && cols_fixed_shape(M, a.L, G, mode)) {
#define SAFR_LAUNCH(m, l, g, md, nn)                \
    if (M == m && a.L == l && G == g && mode == md) \
        return launch_fixed<m, g, l, md, nn>(a, nf, frames, s);
        SAFR_FIXED_SHAPES(SAFR_LAUNCH)
#undef SAFR_LAUNCH
    }
    switch (M) {
        case 32: return launch_generic<32>(a, frames, s);
        case 64: return launch_generic<64>(a, frames, s);
        case 128: return launch_generic<128>(a, frames, s);
        case 256: return launch_generic<256>(a, frames, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace safr
