/*
 * safr.h - C ABI of the MI355X (gfx950) SAFR reconstruction library.
 *
 * SAFR (Weissinger, Hubmer, Stadler, Ramlau; arXiv 2510.19542) solves the
 * atmospheric tomography problem of multi-conjugate adaptive optics with one
 * precomputed per-frequency regularised inverse:
 *
 *   soft real time (Alg. 2): for every spatial frequency n of the M x M grid,
 *     A_n[g, l] = s_l(n) exp(i pi h_l (n_x ax_g + n_y ay_g) / (c_l T))     (Sec. 3.1)
 *     s_l(n)    = gamma_l^(1/2) / c_l (1 + pi^2 |n|^2 / (c_l T)^2)^(-beta/2)
 *     A_n = U S V^H,  B_n[l, g] = s_l(n) sum_r V[l, r] g(S_rr) conj(U[g, r]),
 *     Tikhonov filter g(s) = s / (s^2 + alpha)                              (Sec. 3.1)
 *     (or truncation, a learned filter, and optionally alpha weighted per frequency)
 *   hard real time (Alg. 1): d_g = fft2(Psi_g) for the J guide-star wavefronts,
 *     b_l(n) = sum_g B_n[l, g] d_g(n), Phi_l = ifft2(b_l) for the L layers.
 *
 * Conventions (identical to the CPU reference used by the tests):
 *   - T = M * pitch / 2; layer l's output grid has spacing c_l * pitch and its
 *     index M/2 sits at x = 0 (Sec. 3.2 grids); c_l = 1 (natural stars) or
 *     1 - h_l / h_lgs (laser stars, Sec. 2);
 *   - the n x n pupil data is placed at rows/columns p0 .. p0+n-1 of the M x M
 *     zero grid, p0 = (M - n + 1) / 2 (extension by zero, Sec. 2);
 *   - first array index <-> x <-> ax; arrays are row-major;
 *   - even M: the Nyquist row and column carry B = 0 (symmetric truncation with
 *     m = M/2 - 1 of the frequency index n(j), Sec. 3.2);
 *   - mixed asterisms (both kinds present) use split tomography (Sec. 3.3):
 *     laser-star data has its least-squares tip/tilt plane over the pupil
 *     removed and is reconstructed with alpha; natural-star data is reduced to
 *     that plane and reconstructed with alpha_tt; the natural-star layers are
 *     resampled bilinearly (periodic) onto the laser layer grids and added.
 *
 * Also: the closed-loop step of Alg. 3 (POLC and the integrator around the
 * reconstruction), a Strehl estimate (Marechal, Sec. 4), refreshes of the filter
 * without a new SVD, plan bundles for mixed sizes, an autotuner, and the trainer
 * of the learned filter.
 *
 * Memory: every data pointer passed to a reconstruct call is device memory
 * owned by the caller.  A plan owns B (and the per-frequency SVDs it was built
 * from) and a single-frame workspace.  Calls on a plan are stream ordered on the
 * stream given; reconstruct and loop-step calls neither allocate nor synchronise
 * (unless the debug option SAFR_OPT_CHECK_FINITE is on).  A plan may be used from
 * one thread at a time.
 * No C++ exception crosses this interface; errors are returned as negative
 * safr_status values and described by safr_last_error() (thread local).
 */
#ifndef SAFR_H
#define SAFR_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAFR_OK = 0,
    SAFR_ERR_ARG = -1,          /* null pointer, bad size, bad enum, alpha/beta < 0 */
    SAFR_ERR_GEOMETRY = -2,     /* heights not ascending, h >= h_lgs for laser stars, weights <= 0 */
    SAFR_ERR_DOMAIN = -3,       /* a shifted, scaled aperture leaves c_l Omega_T (Sec. 2) */
    SAFR_ERR_UNSUPPORTED = -4,  /* M not in {32, 64, 128, 256}, n > M, J or L beyond limits */
    SAFR_ERR_NUMERIC = -5,      /* non-finite value in the precomputed operator */
    SAFR_ERR_DEVICE = -6,       /* a HIP runtime call failed */
    SAFR_ERR_STATE = -7         /* workspace too small for the requested frame count */
} safr_status;

enum { SAFR_NGS = 0, SAFR_LGS = 1 };
/* Filters of the regularised inverse (Sec. 3.1):
 *   TIKHONOV  g(s) = s / (s^2 + alpha); alpha = 0: pseudo-inverse (rank tolerance max(G,L) eps s_1);
 *   MLP       learned filter factors (see the learned-filter section below);
 *   TSVD      truncation, g(s) = 1/s for s^2 > alpha (and above the rank tolerance), else 0: the cut
 *             sits where Tikhonov's filter factor s^2 / (s^2 + alpha) is 1/2. */
enum { SAFR_FILTER_TIKHONOV = 0, SAFR_FILTER_MLP = 1, SAFR_FILTER_TSVD = 2 };
enum { SAFR_FP32 = 0, SAFR_BF16X3 = 1 };

#define SAFR_MAX_STARS_PER_GROUP 16
#define SAFR_MAX_LAYERS 16
#define SAFR_MLP_PARAMS 8705

/* One guide star: direction (ax, ay) in radians (Sec. 2) and its kind. */
typedef struct {
    double ax, ay;
    int kind;                       /* SAFR_NGS or SAFR_LGS */
} safr_star;

/* Problem geometry (Sec. 2, Sec. 3.2).  All pointers are host memory, read
 * during safr_precompute only. */
typedef struct {
    int n;                          /* pupil grid n x n, 1 <= n <= M */
    int M;                          /* periodic FFT grid M x M */
    double pitch;                   /* grid spacing [m]; T = M * pitch / 2 */
    int J;                          /* number of guide stars */
    const safr_star* stars;         /* J stars */
    double h_lgs;                   /* sodium layer height [m] (laser stars) */
    const unsigned char* pupil;     /* n*n mask, row-major, nonzero = inside; NULL = all inside */
    double beta;                    /* Sobolev smoothness, >= 0 */
    double alpha_tt;                /* Tikhonov parameter of the natural-star group when mixed */
    int filter;                     /* SAFR_FILTER_TIKHONOV, SAFR_FILTER_MLP or SAFR_FILTER_TSVD */
    const float* mlp;               /* SAFR_MLP_PARAMS network parameters (learned filter only) */
    double noise;                   /* relative noise level, a network input (learned filter only) */
    /* NULL, or [M][M] multipliers w >= 0 of the regularisation parameter per frequency (Sec. 3.1
     * allows one per A_jk): frequency (j, k) uses alpha w[j][k] (alpha_tt w[j][k] for the natural
     * stars of a mixed asterism); j, k are the DFT indices along the first and second grid axis.
     * Must be point-symmetric, w[j][k] = w[(M-j)%M][(M-k)%M], so that B stays Hermitian.
     * Tikhonov and TSVD filters only. */
    const double* alpha_weight;
} safr_geometry;

typedef struct safr_plan safr_plan;

/* Read-only description of a plan (filled by safr_plan_info). */
typedef struct {
    int n, M, J, L;
    int groups;                     /* 1, or 2 for a mixed asterism (group 0 = laser, 1 = natural) */
    int group_size[2];              /* stars per group */
    int group_kind[2];
    double c[SAFR_MAX_LAYERS];      /* output-grid cone coefficients c_l */
    double layer_pitch[SAFR_MAX_LAYERS];   /* c_l * pitch [m] */
    size_t B_complex_per_group[2];  /* stored half-spectrum entries: (M/2+1) * M * L * G */
} safr_plan_desc;

/*
 * Soft-real-time precomputation (Alg. 2, Sec. 3.1): validates the geometry,
 * builds A_n for the half spectrum on the GPU in FP64, takes its SVD (one-sided
 * Jacobi), applies the filter (Tikhonov with alpha, or the learned network of
 * geo->mlp evaluated in BF16 on the features (|n|/(2T), log10 s_r, log10 noise,
 * sum_l gamma_l |V_lr|^2)), and stores B in FP64 (for export), FP32 and BF16
 * hi/lo.  heights[L] [m] ascending, weights[L] > 0 (normalised internally),
 * alpha >= 0 (0 = pseudo-inverse with rank tolerance max(G,L) eps s_1).
 * Allocates device memory and synchronises `stream`.  On success *out owns
 * the plan; release it with safr_destroy.
 */
safr_status safr_precompute(const safr_geometry* geo, int L, const double* heights,
                            const double* weights, double alpha, safr_plan** out,
                            hipStream_t stream);

/*
 * Soft-real-time refresh of the filter (Alg. 2 after its SVD): rebuilds B for new regularisation
 * parameters from the per-frequency SVDs the plan keeps, without recomputing A_n or its SVD.
 * alpha and alpha_tt (natural stars of a mixed asterism; ignored otherwise) >= 0; filter
 * SAFR_FILTER_TIKHONOV or SAFR_FILTER_TSVD (a learned filter is made by safr_precompute);
 * alpha_weight: NULL or host [M][M] multipliers as in safr_geometry.  The natural group and its
 * basis images are rebuilt only when alpha_tt, the filter or a weight map changes, so a change of
 * alpha alone touches only the laser (or only) group.  B, its FP32 copy, the basis images and the
 * BF16 tiles are rewritten in place (pointers, captured graphs and workspaces stay valid): work
 * on `stream` issued before the call uses the old operator, after it the new one; reconstructions
 * on other streams must not run meanwhile.  Synchronises `stream`.  Errors: SAFR_ERR_ARG (bad
 * parameters or map), SAFR_ERR_DEVICE; SAFR_ERR_NUMERIC if a non-finite value appears, after
 * which the plan's operator is undefined (destroy the plan).
 * A refresh that must not hold up a running loop (or a change of the layer weights or of the
 * asterism, which needs safr_precompute) can be built as a second plan on another stream while the
 * current plan keeps serving, and the loop switches plans between two frames.
 */
safr_status safr_update_alpha(safr_plan* p, double alpha, double alpha_tt, int filter, const double* alpha_weight,
                              hipStream_t stream);

/*
 * Hard-real-time reconstruction of one frame (Alg. 1): wavefronts [J][n][n]
 * FP32 device (values outside the pupil are ignored) -> layers [L][M][M] FP32
 * device, layer l on its own grid.  Uses the plan's internal workspace.
 */
safr_status safr_reconstruct(safr_plan* p, const float* wavefronts, float* layers,
                             hipStream_t stream);

/*
 * Batched reconstruction of `frames` independent frames (1..65535, else SAFR_ERR_ARG; SAFR_BF16X3: plans with
 * M <= 128 only, otherwise SAFR_ERR_UNSUPPORTED): wavefronts
 * [frames][J][n][n] -> layers [frames][L][M][M].  precision SAFR_FP32 applies B
 * in FP32; SAFR_BF16X3 applies it on BF16 matrix cores with FP32 accumulation
 * and the split correction B_hi D_hi + B_hi D_lo + B_lo D_hi.  Needs a
 * workspace of safr_workspace_size(p, frames, precision) bytes (internal for
 * frames == 1, else bound with safr_set_workspace) or returns SAFR_ERR_STATE.
 * The launch sequence is captured once per (frames, pointers, precision,
 * stream) into a HIP graph and replayed on later identical calls.
 */
safr_status safr_reconstruct_batched(safr_plan* p, int frames, const float* wavefronts,
                                     float* layers, int precision, hipStream_t stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): safr_reconstruct_batched with the workspace in a static device array of the library
 * (safr_static_workspace_bytes(), 64 MiB; each GPU the library runs on holds its own copy until the process
 * ends) instead of a bound workspace.  Launches the same kernels and gives the same layers; calls no
 * allocating routine and never captures a graph (SAFR_OPT_GRAPH is ignored).  Frame counts whose workspace
 * (safr_workspace_size) exceeds the array are rejected with SAFR_ERR_ARG (MORFEO-like plans: up to 20
 * frames).  Nothing in the path reads the array before writing it, so no call clears it; every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other streams, other threads) race and must
 * be ordered by the caller.  The first call on a device looks up the array's device address (no allocation).
 */
safr_status safr_reconstruct_batched_static(safr_plan* p, int frames, const float* wavefronts, float* layers,
                                            int precision, hipStream_t stream);
size_t safr_static_workspace_bytes(void);

/* Device workspace bytes needed for `frames` frames (1..65535): the row and layer spectra of the call's
 * largest launch sequence (SAFR_OPT_SEQ_FRAMES; about 3 MB per MORFEO-like frame, at most 200 MiB by
 * default) plus, for safr_loop_step, the pseudo-open-loop wavefronts of all its frames.  Depends on the
 * plan's SAFR_OPT_SEQ_FRAMES: a workspace bound before that option is raised may become too small. */
safr_status safr_workspace_size(const safr_plan* p, int frames, int precision, size_t* bytes);

/* Binds caller-owned device memory (>= 256-byte aligned) as the workspace
 * (NULL restores the internal single-frame workspace).  Not owned by the plan. */
safr_status safr_set_workspace(safr_plan* p, void* device_ptr, size_t bytes);

safr_status safr_plan_info(const safr_plan* p, safr_plan_desc* out);

/*
 * Copies the FP64 B of one group to host memory as interleaved (re, im) doubles
 * in the layout [k = 0..M/2][j = 0..M-1][l][g] (k: second frequency index,
 * half spectrum; j: first frequency index).  `count` = number of doubles the
 * buffer holds; must be >= 2 * B_complex_per_group[group].  Synchronises.
 */
safr_status safr_export_B(const safr_plan* p, int group, double* host, size_t count);

/*
 * Replaces the FP64 B of one group by `host` (the layout of safr_export_B, count doubles) and rebuilds
 * what derives from it with the precompute's own arithmetic: the FP32 copy, the BF16 tiles of the
 * matrix-core apply and, for the natural-star group of a mixed asterism, its basis images; a plan that
 * imports another plan's exported B reconstructs exactly as that plan.  The plan's geometry (M, L,
 * stars, pupil) must be the one the B was made for; B must be Hermitian with zero Nyquist row and
 * column (as every exported B is), or the layers are not real.  Restores a refresh of B (Alg. 2 run
 * elsewhere, or saved) without a new SVD; a later safr_update_alpha rebuilds B from the plan's own
 * SVDs again.  Synchronises `stream`.  Errors: SAFR_ERR_ARG (NULL, group, count), SAFR_ERR_NUMERIC
 * (non-finite value), SAFR_ERR_DEVICE.
 */
safr_status safr_import_B(safr_plan* p, int group, const double* host, size_t count, hipStream_t stream);

/* Tuning and execution options of a plan (not needed for correct results):
 *   SAFR_OPT_GRAPH       1 = capture the launch sequence in a HIP graph and replay it
 *                        (non-default streams only), 0 = launch directly (default);
 *   SAFR_OPT_ROW_TEAMS   transform teams per block of the row pass (2 rows per team);
 *   SAFR_OPT_OUT_ROWS    output rows per block of the output pass: 8, 16 or 32, at most M
 *                        and at least 1024 / M (each block transforms (256 / team) / (rows / 2)
 *                        frames at a time; teams are 16 threads at M = 256, 4 at M = 32, 8 else);
 *   SAFR_OPT_OUT_FRAMES  frames per block of the output pass (>= 1; mixed asterisms keep the
 *                        block's natural-star basis pixels in registers across them);
 *   SAFR_OPT_MFMA_FRAMES frames per block of the BF16 apply (4, 8 or 16; default: the
 *                        largest that fits in LDS);
 *   SAFR_OPT_COL_FRAMES  frames per block of the FP32 column pass (>= 1; until set or autotuned it is
 *                        chosen per launch for about two column blocks per CU);
 *   SAFR_OPT_COL_TOGETHER frames the FP32 column pass transforms together (1, 2 or 4; B is
 *                        read once for them; compile-time shapes only, others use 1);
 *   SAFR_OPT_COL_PREFETCH 1 = the column pass uses its compile-time kernel when the shape
 *                        has one (default), 0 = always the generic kernel;
 *   SAFR_OPT_CHECK_FINITE 1 = debug mode: safr_reconstruct(_batched) and safr_loop_step first scan
 *                        their inputs (wavefronts at pupil pixels, the loop's commands everywhere)
 *                        for non-finite values, synchronise the stream, and return SAFR_ERR_NUMERIC
 *                        naming the first such frame without launching the reconstruction; no graph
 *                        is used meanwhile.  Default: 1 if the environment variable SAFR_CHECK_FINITE
 *                        is "1" when the plan is made, else 0 (non-finite inputs then propagate
 *                        within their own frame only);
 *   SAFR_OPT_DEADLINE_US  period P > 0 [us] of the real-time loop (Sec. 1: the loop runs at 500 - 1000 Hz,
 *                        so a step has 1 - 2 ms): every safr_loop_step then stamps the device's
 *                        constant-rate wall clock when the step starts executing and, when its last
 *                        kernel has finished, counts the step and whether it took longer than P (two
 *                        one-thread kernels around the step, captured with it in a graph); read and reset
 *                        the counts with safr_deadline_stats.  0 = off (default).  The first call with
 *                        P > 0 allocates the plan's counters and synchronises;
 *   SAFR_OPT_COL_MFMA    1 = when the FP32 column pass transforms 4 frames together in its
 *                        compile-time kernel, the per-frequency products B_n d_n of those frames run
 *                        on the matrix cores as 4 x 4 x 1 FP32 products (4 layers times the 4 frames,
 *                        one star per step; FP32 products and sums as on the vector units); switching
 *                        it on synchronises the device and lays out a copy of B for it (device memory
 *                        of the size of the column group's FP32 B, padded to multiples of 4 layers).
 *                        0 = on the vector units (default: faster at the configured shapes);
 *   SAFR_OPT_SEQ_FRAMES  frames per launch sequence: a call with more frames runs its row, column and
 *                        output passes for groups of about equal size, one group after the other (the
 *                        tuning options apply per group; results are the same as in one sequence).
 *                        0 = automatic (default): groups whose intermediate spectra take at most
 *                        200 MiB, so that they stay in the GPU's 256 MB Infinity Cache (69 frames at
 *                        MORFEO scale); 1 .. 65535 = at most that many frames per group;
 *   SAFR_OPT_FUSED       1 = FP32 calls of the small configured shape (M = 64, n = 33, one group of 4
 *                        stars, L = 2 or 3) run the whole step of each frame in one block of one kernel,
 *                        its spectra in LDS (default); 0 = the row, column and output passes.  Same
 *                        layers either way.  safr_time_stages then reports the whole step as the row
 *                        stage and zero for the other two.  The closed-loop step uses it too. */
enum { SAFR_OPT_GRAPH = 0, SAFR_OPT_ROW_TEAMS = 1, SAFR_OPT_OUT_ROWS = 2, SAFR_OPT_MFMA_FRAMES = 3,
       SAFR_OPT_COL_FRAMES = 4, SAFR_OPT_COL_PREFETCH = 5, SAFR_OPT_OUT_FRAMES = 6,
       SAFR_OPT_COL_TOGETHER = 7, SAFR_OPT_CHECK_FINITE = 8, SAFR_OPT_DEADLINE_US = 9,
       SAFR_OPT_COL_MFMA = 10, SAFR_OPT_SEQ_FRAMES = 11, SAFR_OPT_FUSED = 12 };
safr_status safr_set_option(safr_plan* p, int option, int value);

/* Deadline monitor of the closed-loop step (SAFR_OPT_DEADLINE_US): steps counted since the last reset,
 * how many took longer than the period, the last and the longest step time.  A step's time runs from
 * when the stream reaches the step to when its output pass has finished (queueing behind earlier work
 * on the stream is not counted).  Synchronises `stream`; reset != 0 zeroes the counts afterwards. */
typedef struct {
    unsigned long long steps, misses;
    double last_us, max_us, period_us;
} safr_deadline_info;
safr_status safr_deadline_stats(safr_plan* p, safr_deadline_info* out, int reset, hipStream_t stream);

/* Measures the three stages of the hard-real-time step (row pass; column pass with the
 * apply; output pass): after one batched call, which leaves every stage's inputs in
 * the workspace, each stage's kernels are launched `iters` times back to back on
 * `stream` between two HIP events; writes the average milliseconds per launch of
 * each to ms[0..2] (a kernel's duration plus the dispatch gap between back-to-back
 * launches), and synchronises `stream` once at the end.  `layers` holds the
 * batched call's result afterwards.  Same buffers and workspace rules as
 * safr_reconstruct_batched. */
safr_status safr_time_stages(safr_plan* p, int frames, const float* wavefronts, float* layers,
                             int precision, int iters, hipStream_t stream, double* ms);

/* Autotuner: for the given frame count and precision, times every admissible
 * row-pass block shape (SAFR_OPT_ROW_TEAMS), output-pass tile and frames per block
 * (SAFR_OPT_OUT_ROWS, SAFR_OPT_OUT_FRAMES) and, for several FP32 frames, column-pass
 * frames per block (SAFR_OPT_COL_FRAMES) with HIP events over `iters` synchronised
 * launches each, and keeps the fastest.  Overwrites `layers`.  choice (may be NULL)
 * receives five ints: row teams, output rows, column frames per block, output frames
 * per block, column frames transformed together. */
safr_status safr_autotune(safr_plan* p, int frames, const float* wavefronts, float* layers, int precision,
                          int iters, hipStream_t stream, int* choice);

/* ---- Closed loop (Alg. 3 without its wavefront-reconstruction step) -------------------------
 * The mirror commands are layers [L][M][M] on the plan's output grids: the layers are placed at
 * the conjugation heights, so no fitting step is needed (Sec. 3.3, Alg. 3).  The tomography
 * operator A of Sec. 2 maps them to each guide star's pupil: (A a)_g at pupil pixel (i, j) is the
 * sum over layers of a_l sampled, by periodic bilinear interpolation, where star g's line of sight
 * through that pixel crosses layer l.  The pixel sits at r = (p0 + i - M/2, p0 + j - M/2) pitch
 * with p0 = (M - n + 1) / 2; the crossing point is c^s_l r + theta_g h_l (c^s_l = 1 - h_l / h_lgs
 * for laser stars, 1 for natural stars), which on layer l's output grid (spacing c_l pitch,
 * centred at index M/2) is the index (c^s_l r + theta_g h_l) / (c_l pitch) + M/2.  Sample
 * positions are evaluated in FP32, values in FP32.
 */

/* POLC (Alg. 3, pseudo-open-loop data) of `frames` frames (1..65535):
 * out[f][g] = pupil .* (wavefronts[f][g] + weight (A layers[f])_g), zero outside the pupil.
 * wavefronts and out [frames][J][n][n], layers [frames][L][M][M], FP32 device memory.  out may
 * be wavefronts (in place); layers must not overlap out.  weight = -1 turns open-loop wavefronts
 * into the residuals a mirror with these commands leaves.  Asynchronous on `stream`.
 * Errors: SAFR_ERR_ARG (NULL, frame count, non-finite weight), SAFR_ERR_DEVICE. */
safr_status safr_polc(safr_plan* p, int frames, const float* wavefronts, const float* layers, float weight,
                      float* out, hipStream_t stream);

/* One time step of Alg. 3 for `frames` independent loops (1..65535), from given closed-loop
 * wavefronts [frames][J][n][n] and the current commands a_in [frames][L][M][M]: POLC
 * (Psi + A a_in), tip/tilt removal of the laser stars and the SAFR reconstruction(s) exactly as
 * safr_reconstruct_batched in FP32, then the integrator a_out = (1 - gain) a_in + gain Phi, fused
 * into the output pass.  a_out may be a_in (in place); neither may overlap wavefronts.  The POLC
 * data lives in the workspace (safr_workspace_size covers it).  With SAFR_OPT_GRAPH the sequence
 * is captured per (frames, pointers, gain, stream) and replayed.  Asynchronous on `stream`.
 * Errors: SAFR_ERR_ARG (NULL, frame count, non-finite gain), SAFR_ERR_STATE (workspace too small),
 * SAFR_ERR_DEVICE. */
safr_status safr_loop_step(safr_plan* p, int frames, const float* wavefronts, const float* a_in, float gain,
                           float* a_out, hipStream_t stream);

/* Strehl estimate in science directions (Sec. 4: Marechal approximation).  For `frames` frames
 * (1..65535) and D directions (1..32; dirs: host [D][2] in rad): the residual phase
 * open_loop[f][d] - A_d(layers[f]) over the pupil, with A_d the operator above for a source at
 * infinity (cone coefficient 1 on every layer), its variance over the pupil pixels after piston
 * removal, times scale^2 (scale converts the data's phase unit to rad at the science wavelength;
 * an empty pupil gives 0), and sr = exp(-variance).  open_loop [frames][D][n][n], layers
 * [frames][L][M][M], sr and var [frames][D], FP32 device memory; var may be NULL.  Directions and
 * sample positions are taken in FP32, the variance is accumulated in FP32 (per 256-pixel chunk,
 * then pairwise merges in a fixed order).  The plan keeps a small buffer of per-chunk moments that
 * grows on demand (the first call with more frames or directions synchronises the stream and
 * allocates); calls on one plan must not overlap.  Otherwise asynchronous on `stream`.
 * Errors: SAFR_ERR_ARG (NULL, counts, non-finite scale or direction), SAFR_ERR_DEVICE. */
safr_status safr_strehl(safr_plan* p, int frames, int D, const double* dirs, const float* open_loop,
                        const float* layers, float scale, float* sr, float* var, hipStream_t stream);

/* ---- Mixed-size batches -------------------------------------------------------------------
 * A bundle of plans (different geometries and grid sizes), each with its own frame count.
 * safr_multi_execute reconstructs every entry's frames (wavefronts[i]: [frames[i]][J][n][n],
 * layers[i]: [frames[i]][L][M][M] of plan i) in one HIP graph launch on `stream`: the first
 * call (and any call with other buffers) captures the entries' launch sequences as parallel
 * branches forked from and joined back to `stream`, later calls replay the graph (on the
 * legacy default stream the sequences are launched directly).  The bundle owns one workspace
 * per entry.  Plans must outlive the bundle; one plan may serve several entries (launches only
 * read it).  Errors: SAFR_ERR_ARG (NULL, count < 1, frames < 1), SAFR_ERR_UNSUPPORTED (BF16X3
 * for a plan without the matrix-core path), SAFR_ERR_DEVICE (allocation, capture, launch). */
typedef struct safr_multi safr_multi;
safr_status safr_multi_create(safr_plan* const* plans, const int* frames, int count, int precision,
                              safr_multi** out);
safr_status safr_multi_execute(safr_multi* m, const float* const* wavefronts, float* const* layers,
                               hipStream_t stream);
/* safr_autotune for every entry with its frame count and buffers (overwrites layers); a plan
 * shared by several entries keeps the choice made for the last of them. */
safr_status safr_multi_autotune(safr_multi* m, const float* const* wavefronts, float* const* layers,
                                int iters, hipStream_t stream);
void safr_multi_destroy(safr_multi* m);

/* ---- Learned spectral filter ------------------------------------------------------------
 * The learned filter replaces Tikhonov's filter factors (Sec. 3.1 admits any regularising
 * filter): g_r = phi_r / s_r for s_r > sqrt(eps) s_1 (else 0),
 * phi = MLP(|n|/(2T), log10 s_r, log10 noise, sum_l gamma_l |V_lr|^2),
 * a 4 -> 64 -> 64 -> 64 -> 1 network (exact GELU, logistic output), SAFR_MLP_PARAMS floats
 * packed W1 (64x4), b1, W2 (64x64), b2, W3, b3, w4 (64), b4 with W[out][in].
 *
 * The trainer is built for one geometry with one kind of guide star.  Frames are generated
 * by the caller as random draws only; the trainer applies the tomography operator in its
 * Fourier form (layer spectra F_l = amp_l z_l, wavefront spectra sum_l exp(2 pi i n . s_gl / M)
 * F_l plus eta sigma_n M z_g, sigma_n the expected wavefront RMS) and stores, per frame and
 * half-spectrum frequency, the statistics of the full-grid layer residual, which is quadratic
 * in phi.  Training minimises the frame-averaged relative residual with Adam, in FP32.
 */
typedef struct safr_trainer safr_trainer;

/* amp: host [L][M/2+1][M] layer amplitudes; room for max_frames frames.  Synchronises. */
safr_status safr_trainer_create(const safr_geometry* geo, int L, const double* heights,
                                const double* weights, const float* amp, int max_frames,
                                safr_trainer** out, hipStream_t stream);
/* zl: device complex64 [count][L][M/2+1][M], zn: device complex64 [count][J][M/2+1][M]
 * (complex normal, E|z|^2 = 1); eta: host [count] noise levels (> 0).  Appends frames. */
safr_status safr_trainer_add_frames(safr_trainer* t, int count, const void* zl, const void* zn,
                                    const float* eta, hipStream_t stream);
/* Copies parameters in (and resets the Adam state) or out (host arrays of SAFR_MLP_PARAMS). */
safr_status safr_trainer_set_params(safr_trainer* t, const float* params);
safr_status safr_trainer_get_params(const safr_trainer* t, float* params);
/* Adam state for checkpoints: first and second moments (host arrays of SAFR_MLP_PARAMS) and the
 * number of steps taken (bias correction).  Set after set_params, which resets the state; the
 * moments must be finite and the second moments >= 0. */
safr_status safr_trainer_get_state(const safr_trainer* t, float* m, float* v, int* step);
safr_status safr_trainer_set_state(safr_trainer* t, const float* m, const float* v, int step);
/* One Adam step (lr; beta1 0.9, beta2 0.999, eps 1e-8) on the frames listed (host indices);
 * loss (may be NULL) receives the batch loss before the step (synchronises when requested). */
safr_status safr_trainer_step(safr_trainer* t, int nb, const int* frames, float lr, double* loss,
                              hipStream_t stream);
/* Gradient of the batch loss with respect to the parameters (host grad, may be NULL), no update. */
safr_status safr_trainer_gradient(safr_trainer* t, int nb, const int* frames, float* grad, double* loss,
                                  hipStream_t stream);
/* The closed-form optimum of the training objective on the listed frames (the same objective as
 * safr_trainer_step's batch loss): it is quadratic in the filter factors at every frequency, so over all
 * filters of the form g_r = phi_r / s_r (the network's, Tikhonov's phi = s^2 / (s^2 + alpha), any other)
 * its minimum is reached at phi* = Qbar^-1 cbar, the statistics summed over the frames (Sec. 3.1 filter
 * functions; components at or below the cutoff sqrt(eps) s_1 get phi = 0).  loss receives the objective
 * at phi*, a lower bound of every network's batch loss on these frames; phi (may be NULL): host [r][H]
 * factors, r = min(J, L), H = (M/2+1) M half-spectrum frequencies h = k M + j.  Synchronises. */
safr_status safr_trainer_optimal_filter(safr_trainer* t, int nb, const int* frames, float* phi, double* loss,
                                        hipStream_t stream);
/* The training objective on the listed frames for Tikhonov's filter, phi = s^2 / (s^2 + alpha) (Sec. 3.1),
 * alpha >= 0.  Synchronises. */
safr_status safr_trainer_tikhonov_loss(safr_trainer* t, int nb, const int* frames, double alpha, double* loss,
                                       hipStream_t stream);
int safr_trainer_frames(const safr_trainer* t);
void safr_trainer_destroy(safr_trainer* t);

/* BF16 inference of the network on device feature rows feats[rows][4] (the third feature is
 * replaced by log10 noise) into device phi[rows]; params on the host.  Synchronises. */
safr_status safr_mlp_infer(const float* params, const float* feats, int rows, double noise, float* phi,
                           hipStream_t stream);

/* Releases the plan and its device memory (NULL is a no-op). */
void safr_destroy(safr_plan* p);

/* Description of the last error on the calling thread (never NULL). */
const char* safr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SAFR_H */
