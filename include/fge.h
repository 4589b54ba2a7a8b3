/*
 * fge.h -- C ABI of the MI355X (gfx950) multi-level foreground estimation library.
 *
 * Method: Germer, Uelwer, Conrad, Harmeling, "Fast Multi-Level Foreground Estimation"
 * (arXiv 2006.14970).  Given an RGB image I and an alpha matte alpha, the library recovers a
 * foreground F and background B with I ~ alpha F + (1 - alpha) B (eq. 1), by Algorithm 1
 * (Section III-D): a coarse-to-fine pyramid of n_l = ceil(log2(max(W, H))) levels of size
 * round(W^(l/n_l)) x round(H^(l/n_l)); at every level the full-resolution I and alpha and the
 * previous level's F, B are resized to the level, then a fixed number of sweeps (10 when the level
 * is at most 32x32, else 2) update every pixel by the closed-form 2x2 solve of eq. 9 -- the
 * compositing data term coupled to the 4 clamped neighbours with weights
 * eps_r + omega |alpha_i - alpha_j| (eq. 3) -- and clamp the result to [0, 1].
 *
 * Choices where the paper is silent: "resize" is nearest-neighbour with source index
 * (x * w_src) / w_dst (integer division); the sweep is red-black (pixels with (x + y) even
 * first, then odd) because the paper's in-place sequential sweep has no parallel form; a 1x1
 * input runs one level.
 *
 * Conventions for every entry point:
 *   - Sizes are passed height first, (H, W), the order of the array shapes below: an image of
 *     H rows of W pixels.  Arrays of sizes (batches) are likewise an array of heights followed by
 *     an array of widths.  The paper writes an input as w x h x 3 (Section III-D); the order of
 *     the arguments here follows the row-major layout, not that notation.
 *   - Images are planar, row-major, x fastest: I, F and B are 3 planes of H*W elements (3 x H x W;
 *     plane c starts at element c*H*W); alpha is one plane of H*W elements (H x W).  Element type
 *     is float32 or IEEE binary16 according to fge_params.storage; values are expected in [0, 1]
 *     and are not checked.
 *   - All data pointers are DEVICE pointers owned by the caller; the library never frees or
 *     keeps them past the call.  F and B must not overlap I, alpha, each other or the workspace:
 *     the estimation entry points compare the byte ranges and return FGE_EINVAL on any overlap.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued asynchronously;
 *     the call returns once it is enqueued.  The caller synchronises before reading F, B.
 *   - Argument errors are reported synchronously (FGE_EINVAL / FGE_EWORKSPACE /
 *     FGE_EUNSUPPORTED) before anything is enqueued; a failed launch returns FGE_EHIP.
 *   - The estimation entry points allocate no device memory: scratch lives in the caller's
 *     workspace (size from fge_workspace_bytes, 256-byte aligned start).
 *   - Arithmetic is float32 on the device for both storage types.  With binary16 storage the
 *     input is read as given and F, B are rounded to binary16 (round to nearest even) once per
 *     level, when a level's state is written to memory.
 */
#ifndef FGE_H
#define FGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fge_status {
    FGE_OK = 0,
    FGE_EINVAL = -1,        /* bad argument (size, pointer, parameter value) */
    FGE_ENOMEM = -2,        /* host allocation failed */
    FGE_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    FGE_EUNSUPPORTED = -4,  /* valid request this build does not implement */
    FGE_EWORKSPACE = -5,    /* workspace missing or smaller than fge_workspace_bytes */
    FGE_EBUDGET = -6,       /* a request that can never fit a server's budget or arena */
    FGE_ECANCELED = -7      /* a server request cancelled before admission */
} fge_status;

/* Element types.  F32 and F16 are storage types of the estimator; U8 (values 0..255 standing
 * for [0, 1]) appears only in the layout conversions below; F64 only in the closed-form solve. */
typedef enum fge_dtype { FGE_F32 = 0, FGE_F16 = 1, FGE_U8 = 2, FGE_F64 = 3 } fge_dtype;

/* Sweep order on the device.  Red-black (pixels with (x + y) even, then odd, each in place) runs
 * on every kernel.  Jacobi (every pixel from the previous sweep's values) runs on per-level
 * kernels only (no coarse block, no fused levels; not in batches or the server).  The paper's
 * sequential raster order exists in the CPU oracle only. */
typedef enum fge_order { FGE_REDBLACK = 0, FGE_JACOBI = 1 } fge_order;

/* Kernel family for the levels above the LDS-resident coarse block. */
typedef enum fge_kernel {
    FGE_KERNEL_AUTO = 0,   /* fused streaming kernel where supported, else per-half-sweep */
    FGE_KERNEL_FUSED = 1,  /* one fused launch per fine level, tile or streaming kernel
                              (requires iters_big == 2) */
    FGE_KERNEL_NAIVE = 2   /* debug path: one launch per resize and per half-sweep */
} fge_kernel;

typedef struct fge_params {
    uint32_t size;          /* sizeof(fge_params), for ABI versioning */
    float omega;            /* alpha-gradient weight omega (Algorithm 1 default 0.1) */
    float eps_r;            /* regulariser eps_r (Algorithm 1 default 5e-3) */
    int32_t small_size;     /* a level is "low resolution" when w <= small and h <= small (32) */
    int32_t iters_small;    /* sweeps on low-resolution levels (10) */
    int32_t iters_big;      /* sweeps on the other levels (2) */
    int32_t storage;        /* fge_dtype of I, alpha, F, B and the workspace state */
    int32_t order;          /* fge_order */
    int32_t kernel;         /* fge_kernel */
    int32_t strip_rows;     /* fused kernel: output rows per wave strip; 0 = automatic */
    int32_t coarse_max_px;  /* levels with w*h <= this (and all smaller ones) run in the
                               LDS-resident coarse kernel (at most 4096); 0 = automatic (the
                               levels up to 1024 px and every level whose sweep count is not 2),
                               -1 = never */
    int32_t tile_max_px;    /* fine levels with w*h <= this use the LDS tile kernel, larger ones
                               the streaming kernel; 0 = automatic (2^18), -1 = never */
} fge_params;

/* Fill *p with the paper's defaults: omega 0.1, eps_r 5e-3, 32 / 10 / 2, float32 storage,
 * red-black order, automatic kernels. */
void fge_default_params(fge_params *p);

/* Human-readable name of a status code (static string). */
const char *fge_status_string(int status);

/* Library ABI version (increments when fge_params or a signature changes); this header is 9
 * (4 moved every size argument to height-first order, 5 added fge_estimate_foreground_noalloc,
 * 6 added the closed-form solve fge_closed_form, 7 the server's failure counters, cancellation
 * and simulated executor, 8 the convergence form in fused passes, 9 fge_level_options.passes). */
int32_t fge_version(void);

/* ---- host-only planning (no GPU needed) ---------------------------------------------- */

/* Level count of Algorithm 1 for an H x W input: ceil(log2(max(W, H))), at least 1.
 * Returns 0 if W or H is outside [1, 32767]. */
int32_t fge_num_levels(int32_t H, int32_t W);

/* Size of level `level` (1-based) of `n_levels` along an axis of `full` pixels:
 * round(full^(level / n_levels)) (Algorithm 1).  Returns 0 on bad arguments. */
int32_t fge_level_size(int32_t full, int32_t level, int32_t n_levels);

/* The level schedule for an H x W input under *p: for l = 1..n, w_out[l-1], h_out[l-1] and
 * iters_out[l-1] (10 or 2 by the low-resolution rule), and *n_coarse_out, the number of leading
 * levels the LDS-resident coarse kernel runs.  Arrays hold at least max_levels entries (16 is
 * always enough).  FGE_EINVAL on bad sizes or parameters. */
fge_status fge_plan(int32_t H, int32_t W, const fge_params *p, int32_t max_levels,
                    int32_t *w_out, int32_t *h_out, int32_t *iters_out, int32_t *n_levels_out,
                    int32_t *n_coarse_out);

/* Workspace bytes fge_estimate_foreground needs for an H x W input under *p (0 on bad
 * arguments; may be 0 for inputs whose pyramid fits the coarse kernel). */
size_t fge_workspace_bytes(int32_t H, int32_t W, const fge_params *p);

/* ---- estimation ------------------------------------------------------------------------ */

/* Algorithm 1 for one image: reads I (3 x H x W) and alpha (H x W), writes F and B
 * (3 x H x W each), all in p->storage element type, on `stream`.  `workspace` must hold
 * fge_workspace_bytes(H, W, p) bytes (it may be NULL when that is 0).  p == NULL means the
 * defaults.  Before the finest level writes them, the call may use F's memory for compact
 * copies of the lower levels' inputs, so F and B must not overlap I, alpha or the workspace
 * (as for any output). */
fge_status fge_estimate_foreground(const void *I, const void *alpha, int32_t H, int32_t W,
                                   const fge_params *p, void *F, void *B, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* The same computation as fge_estimate_foreground with no workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a file-scope device array of
 * FGE_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, held from the first call on
 * that device until the process ends; the call allocates nothing, host or device.  It runs on
 * the device current at the call (which must be `stream`'s device).  Results are bit-identical
 * to fge_estimate_foreground's under the same parameters.  Inputs whose fge_workspace_bytes
 * exceeds FGE_NOALLOC_SCRATCH_BYTES are rejected with FGE_EWORKSPACE (at a 4:3 aspect that
 * admits images up to about 8.3 MP in float32 and 15.6 MP in binary16 storage: 4096 x 3072 fits
 * in binary16 only);
 * order FGE_JACOBI is FGE_EUNSUPPORTED.  Every call on a device shares that device's array and
 * leaves its contents behind: calls that overlap in time on one device (different streams, or
 * threads whose launches are not ordered) race and give undefined results. */
#define FGE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fge_status fge_estimate_foreground_noalloc(const void *I, const void *alpha, int32_t H, int32_t W,
                                           const fge_params *p, void *F, void *B, void *stream);

/* Algorithm 1's "while not converged" form on the fused kernels, the test taken after every pass
 * of two sweeps: every level runs passes of two sweeps in p->order (one memory round trip each:
 * the LDS tile kernel for levels up to p->tile_max_px, the streaming kernel above; the first pass
 * resizes from the previous level), and stops when a pass changes the level's energy (fge_energy's
 * quadratic on the level's F, B against its nearest-resized image and matte) by at most tol times
 * its value before the pass -- before the first pass: the previous level's result as the resize
 * leaves it -- or after max_passes passes (1..100000).  Each level thus runs an even number of
 * sweeps; the CPU oracle's fgo_ml_converge_every with m = 2 is the same loop.  The leading
 * levels that fit the coarse block (w*h <= p->coarse_max_px, or up to 4096 px when it is 0; none
 * when it is -1) run in one workgroup that reduces each energy in float64 and takes the decision
 * itself.  For the other levels the energies are reduced on the device and read by the host,
 * which keeps passes in flight beyond the one it judges (each writes another state buffer, so
 * the accepted state is never overwritten): the call BLOCKS until the result is complete.  passes_out (HOST int array of >= n_levels
 * entries, or NULL) receives the passes each level ran.  The state stays float32 between passes
 * and levels (float16 inputs are converted once) and F, B are written in p->storage at the end.
 * In the Jacobi order every level runs on the tile kernel (each sweep from the state before it,
 * in LDS) and none in the coarse block, which is red-black.  Workspace:
 * fge_converge_passes_workspace_bytes (three float32 states at full size, about 72 B/px, plus
 * 16 B/px of float32 inputs in float16 storage, plus the float32 inputs of the largest level
 * below full size, about 4 B/px). */
size_t fge_converge_passes_workspace_bytes(int32_t H, int32_t W, const fge_params *p);
fge_status fge_estimate_foreground_converge_passes(const void *I, const void *alpha, int32_t H,
                                                   int32_t W, const fge_params *p, double tol,
                                                   int32_t max_passes, void *F, void *B,
                                                   int32_t *passes_out, void *workspace,
                                                   size_t workspace_bytes, void *stream);

/* Algorithm 1's level loop in its "while not converged" form: at every level, after the resize,
 * sweep (in p->order) until the level's energy -- fge_energy's quadratic on the level's F, B
 * against its nearest-resized image and matte -- changes by at most tol times its value before
 * the sweep, or until max_sweeps sweeps (1..100000) have run; at least one sweep runs.  The
 * energy is reduced and the decision taken on the device after every sweep: the call enqueues
 * max_sweeps sweeps per level and returns at once, and the launches after convergence do nothing.
 * tol < 0 runs the fixed counts of the iteration rule instead (max_sweeps ignored).  sweeps_out
 * (DEVICE int array of >= n_levels entries, or NULL) receives the sweeps each level ran (in the
 * tol >= 0 form).  Every level runs on per-level kernels (no coarse block, no fused levels), so
 * this is a quality mode, not the fast path.  Workspace: fge_converge_workspace_bytes. */
size_t fge_converge_workspace_bytes(int32_t H, int32_t W, const fge_params *p);
fge_status fge_estimate_foreground_converge(const void *I, const void *alpha, int32_t H, int32_t W,
                                            const fge_params *p, double tol, int32_t max_sweeps,
                                            void *F, void *B, int32_t *sweeps_out, void *workspace,
                                            size_t workspace_bytes, void *stream);

/* Resize variant of the pyramid (the paper does not name the kernel).  NEAREST is the reading
 * used everywhere; SMOOTH area-averages the full-resolution image and matte to every level (each
 * level pixel is the overlap-weighted mean of its footprint) and resizes the previous level's F
 * and B bilinearly (pixel centres at half-integers, clamped at the borders). */
typedef enum fge_resize { FGE_RESIZE_NEAREST = 0, FGE_RESIZE_SMOOTH = 1 } fge_resize;

typedef struct fge_level_options {
    uint32_t size;         /* sizeof(fge_level_options) */
    int32_t resize;        /* fge_resize */
    double tol;            /* < 0: the fixed sweep counts; >= 0: the convergence form above */
    int32_t max_sweeps;    /* convergence form: 1..100000 sweeps (passes) per level */
    int32_t passes;        /* 0: the test after every sweep, on per-level kernels; 1: the form of
                              fge_estimate_foreground_converge_passes (tol >= 0, the test
                              after every pass of two sweeps on the fused kernels, max_sweeps caps
                              the passes and sweeps_out receives them; the call returns when the
                              result is complete) with this resize variant; with SMOOTH no coarse
                              block runs (its resize is the nearest map) */
} fge_level_options;

/* The level loop with these options (order from p->order): the general form of
 * fge_estimate_foreground_converge (which is resize NEAREST), on per-level kernels.  The smooth
 * variant's level inputs are float32 copies (area sums in float64).  One exception: the smooth
 * variant with the red-black order and fixed counts (tol < 0, kernel not FGE_KERNEL_NAIVE) runs a
 * level's sweeps on the fused kernels, in passes of two sweeps between two float32 state buffers
 * (plus one per-level sweep for an odd count); the same sweeps in another rounding order.
 * Workspace: fge_levels_workspace_bytes (that case adds a second float32 state and, for binary16
 * storage, float32 copies of I and alpha: 16 bytes per pixel). */
size_t fge_levels_workspace_bytes(int32_t H, int32_t W, const fge_params *p,
                                  const fge_level_options *o);
fge_status fge_estimate_foreground_levels(const void *I, const void *alpha, int32_t H, int32_t W,
                                          const fge_params *p, const fge_level_options *o,
                                          void *F, void *B, int32_t *sweeps_out, void *workspace,
                                          size_t workspace_bytes, void *stream);

/* ---- closed-form global solve (Section III-B, eq. 2) ----------------------------------- */

/* The closed-form estimate the paper compares against (Section III-B): the minimiser of eq. 2,
 * per colour channel
 *   sum_i (a_i F_i + (1 - a_i) B_i - I_i)^2
 *     + sum over horizontal and vertical neighbour pairs {i, j} of
 *       w_ij ((F_i - F_j)^2 + (B_i - B_j)^2),   w_ij = eps + omega |a_i - a_j|,
 * with eq. 2's gradient magnitudes |alpha_x|, |alpha_y| read as forward differences.  omega = 1
 * is eq. 2 as printed; eps > 0 is the regulariser of Section III-C, without which F is free where
 * alpha = 0 and B where alpha = 1 (the system is then singular).  No clamp: the unconstrained
 * minimiser.  The 2n x 2n normal equations A x = b (x_i = (F_i, B_i), the same A for the three
 * channels) are solved by conjugate gradients with a block-Jacobi preconditioner (the exact
 * inverse of A's 2x2 diagonal blocks; the paper's remark after eq. 2 uses a thresholded
 * incomplete Cholesky factor, whose triangular solves are sequential), in float64 on the device,
 * until every channel's relative residual |b - A x| / |b| is at most tol (the remark quotes
 * 1e-6) or max_iter iterations have run.  A is positive definite unless alpha is constant over
 * the whole image. */
typedef struct fge_cf_params {
    uint32_t size;        /* sizeof(fge_cf_params) */
    int32_t storage;      /* fge_dtype of I, alpha, F, B: FGE_F32, FGE_F16 or FGE_F64 */
    double omega;         /* weight of |alpha_i - alpha_j| (1.0, eq. 2) */
    double eps;           /* regulariser added to every edge weight, > 0 (5e-3, Section III-C) */
    double tol;           /* relative residual per channel, > 0 (1e-6) */
    int32_t max_iter;     /* iteration cap, 0..1000000; 0 = 20000 */
    int32_t warm_start;   /* 1: start from the F, B the output buffers hold; 0: from zero */
} fge_cf_params;

typedef struct fge_cf_info {
    int32_t iterations;            /* iterations of the slowest channel */
    int32_t converged;             /* 1 when every channel reached tol */
    int32_t channel_iterations[3]; /* iterations each channel ran until it converged */
    int32_t breakdown;             /* 1 if a search direction had p.Ap <= 0 (singular A) */
    double rel_residual[3];        /* |b - A x~| / |b| of the stored F, B (x~: x rounded to the
                                      storage type), recomputed after the last iteration */
    double recursive_rel_residual[3]; /* the CG recurrence's own residual at its stop */
    double device_ms;              /* event time on `stream` from the start of the first kernel
                                      to the end of the last (includes the launches enqueued
                                      after convergence, which return at once) */
} fge_cf_info;

/* Fill *p with the defaults above (omega 1, eps 5e-3, tol 1e-6, 20000 iterations, float32). */
void fge_cf_default_params(fge_cf_params *p);

/* Workspace bytes of fge_closed_form for an H x W input (0 on bad sizes): five float64 vectors of
 * 6 planes (x, r, two search directions, A p) plus scalars and partial sums, about 240 B/px. */
size_t fge_cf_workspace_bytes(int32_t H, int32_t W);

/* Solve for F, B (3 x H x W each) from I (3 x H x W) and alpha (H x W), all device buffers in
 * p->storage type (p == NULL: the defaults), on `stream`.  Unlike the estimation calls this one
 * BLOCKS the calling thread until the solve has finished on the device: the iteration count
 * depends on the data, so the host enqueues iterations in chunks and reads a device flag
 * between them (pinned host memory and two events are created per call; no device memory is
 * allocated).  *info (may be NULL) receives the iteration counts and residuals.  FGE_EINVAL on
 * bad sizes (H * W >= 2 is required), parameters, or outputs overlapping the inputs or the
 * workspace; FGE_EWORKSPACE if the workspace is missing, unaligned or smaller than
 * fge_cf_workspace_bytes; FGE_ENOMEM if the pinned host words cannot be allocated. */
fge_status fge_closed_form(const void *I, const void *alpha, int32_t H, int32_t W,
                           const fge_cf_params *p, void *F, void *B, void *workspace,
                           size_t workspace_bytes, void *stream, fge_cf_info *info);

/* ---- batches of images of different sizes ---------------------------------------------- */

/* A batch plan: every image runs Algorithm 1 (Section III-D) on its own level plan -- the level
 * sizes round(W^(l/n_l)) x round(H^(l/n_l)), 10 sweeps on low-resolution levels and 2 on the
 * others, the per-pixel solve of eq. 9 -- so its F and B are bit-identical to
 * fge_estimate_foreground's, and the levels of all images are aligned from the finest.  A run
 * is: one upload of descriptor tables into the workspace, a counter fill kernel, one batched
 * gather pre-pass, one batched coarse block (a workgroup per image), then per fine step one
 * persistent tile-kernel launch and one persistent streaming-kernel launch whose waves pull
 * (level, tile|strip) items from a per-step work queue.  Requires the coarse block (coarse_max_px
 * != -1) and fused fine levels (iters_big == 2, kernel != FGE_KERNEL_NAIVE). */
typedef struct fge_batch fge_batch;

/* Plan a batch of n images, image i of H[i] rows of W[i] pixels, all under *p (NULL =
 * defaults).  Host-only; *out receives the plan.  FGE_EINVAL / FGE_EUNSUPPORTED on bad input. */
fge_status fge_batch_create(int32_t n, const int32_t *H, const int32_t *W, const fge_params *p,
                            fge_batch **out);

/* Release the plan (waits for its last descriptor upload and for the last replay of its graph). */
void fge_batch_destroy(fge_batch *b);

/* Workspace bytes a run of this plan needs (state buffers, compact copies, tables, counters). */
size_t fge_batch_workspace_bytes(const fge_batch *b);

/* Number of aligned fine steps, and of kernel launches (plus one copy) per run. */
int32_t fge_batch_steps(const fge_batch *b);
int32_t fge_batch_launch_count(const fge_batch *b);

/* Run the batch: I[i], alpha[i], F[i], B[i] are image i's device buffers (layout and type as in
 * fge_estimate_foreground; F[i] and B[i] must not overlap any image's inputs or the workspace).  Asynchronous on `stream`; the descriptor tables are uploaded from a
 * pinned staging buffer owned by the plan, and a second run first waits for the previous run's
 * upload (not its kernels).  The plan must not be used by two threads at once. */
fge_status fge_batch_run(fge_batch *b, const void *const *I, const void *const *alpha,
                         void *const *F, void *const *B, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Capture one run with these pointers into a hipGraph owned by the plan (stream must not be
 * NULL); fge_batch_replay launches it again on any stream.  Nothing is executed by the capture.
 * Replays of one plan run one after the other (a replay on another stream first waits for the
 * previous one: they share the workspace).  A new capture first waits for every replay of the
 * previous graph to finish (it rewrites the pinned table buffer the graph's upload node reads),
 * then replaces that graph. */
fge_status fge_batch_capture(fge_batch *b, const void *const *I, const void *const *alpha,
                             void *const *F, void *const *B, void *workspace,
                             size_t workspace_bytes, void *stream);
fge_status fge_batch_replay(fge_batch *b, void *stream);

/* One-shot forms: workspace size for, and a run of, a batch planned on the fly. */
size_t fge_batch_workspace_bytes_for(int32_t n, const int32_t *H, const int32_t *W,
                                     const fge_params *p);
fge_status fge_estimate_foreground_batch(int32_t n, const void *const *I, const void *const *alpha,
                                         const int32_t *H, const int32_t *W, const fge_params *p,
                                         void *const *F, void *const *B, void *workspace,
                                         size_t workspace_bytes, void *stream);

/* ---- reporting and layout ------------------------------------------------------------- */

/* Energy of a result, reduced on the device in float64 (deterministic order):
 *   E = sum_i sum_c (a_i F_i^c + (1 - a_i) B_i^c - I_i^c)^2
 *     + sum over undirected in-bounds 4-neighbour edges {i,j}, each once, of
 *       (eps_r + omega |a_i - a_j|) sum_c [(F_i^c - F_j^c)^2 + (B_i^c - B_j^c)^2],
 * the quadratic whose per-pixel stationarity conditions are the systems of eq. 9 (eq. 3's local
 * costs with each edge counted once), plus the compositing residual |aF + (1-a)B - I| (eq. 1) over
 * the fractional pixels 0 < a < 1.  All buffers are device buffers in p->storage type (H x W
 * planes as for fge_estimate_foreground); p supplies omega, eps_r and the storage type (NULL =
 * defaults).  `out` is a DEVICE array of 6 doubles: E, the data term, the smoothness term, the mean
 * and the max |residual| over fractional pixels, and their count.  The workspace (256-byte
 * aligned) holds fge_energy_workspace_bytes(H, W) bytes of partial sums.  Asynchronous. */
size_t fge_energy_workspace_bytes(int32_t H, int32_t W);
fge_status fge_energy(const void *I, const void *alpha, const void *F, const void *B, int32_t H,
                      int32_t W, const fge_params *p, double *out, void *workspace,
                      size_t workspace_bytes, void *stream);

/* The paper's error measures of a foreground estimate F against a reference G (Section IV,
 * "Error Measures"): over
 * the translucent pixels 0 < a_i < 1 of the reference matte `alpha`, each weighted by a_i,
 *   SAD = sum a_i |F_i - G_i|_1,  MSE = sum a_i |F_i - G_i|_2^2,
 *   GRAD = sum a_i |grad F_i - grad G_i|_2^2,
 * gradients from first-order Gaussian derivative filters of standard deviation `sigma` (the
 * paper's 1.4): the sampled Gaussian of radius int(4 sigma + 0.5) <= 16, normalised to sum 1,
 * times x / sigma^2 along the derivative axis, with mirrored borders, for x and y and every
 * channel.  F, G (3 planes) and alpha (1 plane) are H x W device buffers of type dtype (F32 or
 * F16).  `out` is a DEVICE array of 4 doubles: SAD, MSE, GRAD and the number of translucent
 * pixels.  All arithmetic in float64; the reduction order is fixed.  Workspace:
 * fge_quality_workspace_bytes (256-byte aligned). */
size_t fge_quality_workspace_bytes(int32_t H, int32_t W);
fge_status fge_quality(const void *F, const void *G, const void *alpha, int32_t H, int32_t W,
                       int32_t dtype, double sigma, double *out, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Composite onto a new background (eq. 1 used forward): C = alpha F + (1 - alpha) B, computed in
 * float64 (each product and the sum rounded once) and rounded to dtype.  Planar device buffers. */
fge_status fge_composite(const void *F, const void *alpha, const void *B, int32_t H, int32_t W,
                         int32_t dtype, void *C, void *stream);

/* Interleaved H x W x C images (C = 3: RGB, or 4: RGBA) to planar: 3 colour planes into `planes`
 * and, for C = 4, the fourth channel into `alpha` (one plane).  Element types are fge_dtype
 * values: U8 maps v to v / 255 (float32 division); a float maps to U8 as
 * round-half-even(clamp(v, 0, 1) * 255); F32 -> F16 rounds to nearest even.  Device buffers. */
fge_status fge_hwc_to_planar(const void *src, int32_t src_dtype, int32_t channels, int32_t H,
                             int32_t W, void *planes, void *alpha, int32_t dst_dtype, void *stream);
/* Planar 3 x H x W to interleaved H x W x 3, with the same conversions. */
fge_status fge_planar_to_hwc(const void *planes, int32_t src_dtype, int32_t H, int32_t W,
                             void *dst, int32_t dst_dtype, void *stream);

/* ---- autotuner ------------------------------------------------------------------------- */

/* The autotuner times candidate execution settings of one workload on the device and returns
 * the fastest as a full fge_params (the caller's other fields kept).  It searches the two
 * settings that change how the work is cut, never what is computed: strip_rows (the streaming
 * kernel's strip height, i.e. how many output rows share the halo of the two fused sweeps; 0 is
 * the automatic choice) over {0, 16, 24, 32, 48, 64, 96}, and tile_max_px (the largest level on
 * the LDS tile kernel) over {2^16, 2^18, 2^20}: fge_tune_candidates() settings.  Each runs
 * once untimed, then `reps` times (0 = 3) between two events on `stream`; the call blocks until
 * the search is done.  F and B hold the last candidate's result (all candidates agree to the
 * parity tolerance).  entries[k] (k < max_entries) receives each candidate's strip_rows,
 * tile_max_px, mean milliseconds and status; *n_entries the number of candidates run.  The
 * workspace must hold fge_tune_workspace_bytes (the largest of the candidates' needs).  Callers
 * keep the result (e.g. keyed by device, sizes and storage) and pass it to later calls. */
typedef struct fge_tune_entry {
    int32_t strip_rows;
    int32_t tile_max_px;
    float ms;
    int32_t status;
} fge_tune_entry;

int32_t fge_tune_candidates(void);
size_t fge_tune_workspace_bytes(int32_t H, int32_t W, const fge_params *p);
fge_status fge_autotune(const void *I, const void *alpha, int32_t H, int32_t W, const fge_params *p,
                        void *F, void *B, void *workspace, size_t workspace_bytes, void *stream,
                        int32_t reps, fge_params *best, fge_tune_entry *entries,
                        int32_t max_entries, int32_t *n_entries);

/* The same search for a batch: each candidate is a batch plan (fge_batch_create) run with
 * fge_batch_run.  The workspace must hold fge_batch_tune_workspace_bytes. */
size_t fge_batch_tune_workspace_bytes(int32_t n, const int32_t *H, const int32_t *W,
                                      const fge_params *p);
fge_status fge_batch_autotune(int32_t n, const void *const *I, const void *const *alpha,
                              const int32_t *H, const int32_t *W, const fge_params *p,
                              void *const *F, void *const *B, void *workspace,
                              size_t workspace_bytes, void *stream, int32_t reps, fge_params *best,
                              fge_tune_entry *entries, int32_t max_entries, int32_t *n_entries);

/* ---- serving: continuous batching of requests that arrive over time -------------------- */

/* A server runs requests (one image each, Algorithm 1 as fge_estimate_foreground runs it, so a
 * request's F and B are bit-identical to that call's) on one stream with continuous batching at
 * level granularity.  A scheduler thread owned by the server repeats a "tick": it admits queued
 * requests in arrival order while the HBM budget and the slot count allow, then enqueues ONE
 * set of batched launches (the gather and coarse kernels for the requests admitted in this tick,
 * then one persistent tile launch and one persistent streaming launch) that advances EVERY
 * admitted request by one fine level; a new request also runs its first fine level in the tick
 * that admits it.  So requests that arrive while others are on the device join the next tick and
 * share its launches; each request's pyramid state (its intermediate levels' F and B and the
 * compact input copies) stays in its own block of the server's arena from admission to
 * completion.  Ticks are enqueued up to pipeline_depth ahead of the device.
 *
 * Memory.  The caller hands the server one device arena.  It holds the tick tables
 * (fge_server_reserved_bytes) and every admitted request's workspace, carved first-fit.  The
 * budget bounds the sum of admitted requests' footprints, fge_server_request_bytes: their I,
 * alpha, F and B (caller buffers, held by the request until it completes) plus the workspace.
 * A request is admitted only when both its footprint fits the budget and its workspace fits the
 * arena; it is released when the device has finished its last level.
 *
 * Timing.  At creation the server records a start event on its idle stream; a request's ready
 * time is the device timestamp of the end of its last tick, and its latency is that minus its
 * submission time on the host's steady clock, both relative to the start event. */
typedef struct fge_server fge_server;

typedef struct fge_server_config {
    uint32_t size;             /* sizeof(fge_server_config) */
    int32_t max_active;        /* most requests admitted at once; 0 = 1024 */
    int32_t pipeline_depth;    /* ticks enqueued ahead of the device (1..8); 0 = 2 */
    int32_t reserved0;
    uint64_t budget_bytes;     /* bound on the admitted footprints; 0 = the arena size */
    uint64_t tick_table_bytes; /* descriptor and work-list capacity of one tick; 0 = 16 MiB */
} fge_server_config;

typedef struct fge_server_result {
    int64_t id;                /* the id given to fge_server_submit */
    int32_t status;            /* FGE_OK, or the error that ended the server */
    int32_t ticks;             /* ticks the request took part in */
    double submit_ms;          /* host submission time, ms after the start event */
    double admit_ms;           /* host time the scheduler admitted it */
    double ready_ms;           /* device time its F and B were complete */
    double latency_ms;         /* ready_ms - submit_ms */
} fge_server_result;

typedef struct fge_server_stats {
    int64_t submitted, completed, ticks, launches;   /* completed counts every result, failed
                                                        and cancelled ones too */
    int64_t mixed_ticks;       /* ticks that advanced requests at two or more different levels */
    int64_t admitted_while_busy; /* requests admitted while other requests were on the device */
    int32_t peak_active;
    int32_t reserved0;
    uint64_t peak_charged_bytes; /* peak sum of admitted footprints (<= budget_bytes) */
    uint64_t peak_arena_bytes;   /* peak arena bytes in use (tables included) */
    double mean_active;        /* admitted requests per tick, averaged over ticks */
    int64_t failed;            /* requests completed with an error */
    int64_t cancelled;         /* requests cancelled before admission */
} fge_server_stats;

/* Fill *c with the defaults above. */
void fge_server_default_config(fge_server_config *c);

/* Footprint an H x W request is charged against the budget under *p (0 on bad arguments). */
size_t fge_server_request_bytes(int32_t H, int32_t W, const fge_params *p);

/* Arena bytes the server keeps for its tick tables under *c (the rest holds workspaces). */
size_t fge_server_reserved_bytes(const fge_server_config *c);

/* Create a server for requests under *p (NULL = defaults; the same restrictions as batches:
 * coarse block and fused fine levels) and *c (NULL = defaults).  `arena` is a device buffer of
 * arena_bytes (256-byte aligned start), owned by the caller, which must keep it alive and unused
 * until fge_server_destroy returns.  `stream` (not NULL) is the hipStream_t every launch goes to.
 * Starts the scheduler thread.  Allocates pinned host staging and events, no device memory. */
fge_status fge_server_create(const fge_params *p, const fge_server_config *c, void *arena,
                             size_t arena_bytes, void *stream, fge_server **out);

/* Queue a request: I (3 x H x W), alpha (H x W), F and B (3 x H x W) are device buffers in
 * p->storage type, laid out as for fge_estimate_foreground, ready when this is called (the
 * server's stream does not wait for other streams), and left alone by the caller until the
 * request is reported complete.  Returns at once.  FGE_EBUDGET if the request could never be
 * admitted; FGE_EINVAL / FGE_EUNSUPPORTED on bad arguments; FGE_EHIP if the server has failed. */
fge_status fge_server_submit(fge_server *s, int64_t id, const void *I, const void *alpha,
                             int32_t H, int32_t W, void *F, void *B);

/* Cancel a request that is still queued (submitted, not yet admitted): it completes at once with
 * status FGE_ECANCELED and is reported by fge_server_poll like any other.  FGE_EINVAL if no
 * queued request has this id (unknown, already admitted -- it then runs to completion -- or
 * completed). */
fge_status fge_server_cancel(fge_server *s, int64_t id);

/* Move up to `cap` completed requests (completion order) into out[]; returns how many, or a
 * negative status if the server has failed.  Never blocks.  A request's status is FGE_OK, the
 * error of a tick whose launch failed (FGE_EHIP: that tick's requests fail, the server goes on),
 * FGE_ECANCELED, or the error that ended the server (an error of the device itself: every request
 * not yet completed fails with it). */
int32_t fge_server_poll(fge_server *s, fge_server_result *out, int32_t cap);

/* Block until every request submitted so far has completed (results stay pollable). */
fge_status fge_server_drain(fge_server *s);

/* Counters since creation. */
fge_status fge_server_get_stats(fge_server *s, fge_server_stats *out);

/* Drain, stop the scheduler thread and free the server's host resources (not the arena). */
void fge_server_destroy(fge_server *s);

/* A server whose device is a host model, for testing schedules without a GPU and under host
 * sanitizers: the same scheduler (admission, budget, tick tables, failures, cancellation) drives
 * a simulated executor that uploads and launches nothing and touches no buffer -- the arena is a
 * reserved range of the address space and request pointers are only stored.  A tick takes
 * us_per_launch per launch (the upload counts as one) plus us_per_mpx per megapixel of the fine
 * levels it advances; ticks run one after another.  Failure injection: the k-th tick's launch
 * fails (fail_launch_tick = k; its requests fail with FGE_EHIP, the server goes on), or the k-th
 * tick reports a device error when it completes (fail_device_tick = k; the server fails).
 * manual = 1: no scheduler thread and a clock that only moves when the caller calls
 * fge_server_sim_step, so a schedule is reproducible exactly; fge_server_drain and
 * fge_server_destroy then step the server themselves until every request has completed.
 * manual = 0: a scheduler thread and the host clock, as with the HIP executor. */
typedef struct fge_server_sim {
    uint32_t size;             /* sizeof(fge_server_sim) */
    int32_t manual;            /* 1 (default): stepped by the caller; 0: own thread */
    double us_per_launch;      /* modelled time per launch (3.0) */
    double us_per_mpx;         /* modelled time per megapixel of fine levels (8.0) */
    int32_t fail_launch_tick;  /* 0 = none */
    int32_t fail_device_tick;  /* 0 = none */
} fge_server_sim;

void fge_server_sim_default(fge_server_sim *m);
fge_status fge_server_create_simulated(const fge_params *p, const fge_server_config *c,
                                       size_t arena_bytes, const fge_server_sim *m,
                                       fge_server **out);

/* Manual mode: advance the clock by advance_ms, complete the `complete` oldest ticks in flight
 * (at the later of their modelled end and the clock), then run the scheduler until it has
 * nothing more to enqueue.  Returns the ticks enqueued, or a negative status (the error that
 * ended the server, FGE_EINVAL for bad arguments or a server not in manual mode). */
int32_t fge_server_sim_step(fge_server *s, int32_t complete, double advance_ms);

/* Ticks of a simulated server launched and not yet completed (manual) or reported (thread). */
int32_t fge_server_sim_inflight(fge_server *s);

/* ---- profiling ------------------------------------------------------------------------- */

/* Start recording HIP events around every kernel launch of the following estimation calls
 * (on the caller's stream).  Level 0 is the finest level, 1 the next coarser, ...; the coarse
 * kernel is recorded under the index of the last level it runs, and the gather pre-pass (the
 * compact copy of the small levels' inputs) under index n_levels.  `capacity` bounds the number
 * of recorded launches (events are created here, not in the estimation calls). */
fge_status fge_profile_start(int32_t capacity);

/* Stop recording, wait for the recorded events and report, for each level index below
 * max_levels, the summed milliseconds and the number of launches recorded.  Frees the events. */
fge_status fge_profile_stop(double *level_ms, int32_t *level_launches, int32_t max_levels);

#ifdef __cplusplus
}
#endif

#endif /* FGE_H */
