// Internal declarations shared by the planner, the kernels and the C ABI of libfge.
#pragma once

#include <cstddef>
#include <cstdint>

#include "fge.h"

namespace fge {

constexpr int kMaxLevels = 16;         // 32767 needs 15 levels
constexpr int kMaxSide = 32767;        // keeps x * w_src inside int32
constexpr int kCoarseMaxPx = 4096;     // LDS-resident coarse levels: 2 float4 per pixel = 128 KB
constexpr int kCoarseAutoPx = 1024;    // automatic coarse limit (plus all low-resolution levels)
constexpr int kCoarseThreads = 512;
constexpr int kCoarsePairsPerThread = 4;   // a coarse level has at most 2048 pixel pairs
constexpr int kCoarseMaxPairs = kCoarseThreads * kCoarsePairsPerThread;

enum LevelKind { kKindCoarse = 0, kKindStream = 1, kKindTile = 2, kKindNaive = 3 };
constexpr long kTileMaxPxDefault = 1L << 18;   // fine levels up to 256K px use the tile kernel
constexpr long kGatherMaxPx = 1L << 16;        // coarse/tile levels up to 64K px read a compact copy

struct Level {
    int w, h, iters;
};

// The level schedule of Algorithm 1 plus the execution layout chosen for it.
struct Plan {
    int W = 0, H = 0;
    int n = 0;      // number of levels
    int nc = 0;     // levels [0, nc) run inside the coarse kernel
    Level lv[kMaxLevels];
    int elem = 4;   // bytes per stored element
    // Two ping-pong state buffers in the workspace.  Each holds F (3 planes) then B (3 planes)
    // of one level at that level's size.  A stored level i < n-1 lives in buffer buf_of[i]
    // (the stored levels alternate from the last one down; -1: not stored); the last level is
    // written straight into the caller's F and B.
    size_t buf_off[2] = {0, 0};
    size_t buf_px[2] = {0, 0};
    int buf_of[kMaxLevels] = {};
    size_t ws_bytes = 0;
    int kind[kMaxLevels] = {};     // per fine level: a LevelKind
    // Gather: the ng levels with copy[i] set get a compact copy of their resized I (3 planes)
    // and alpha (1 plane) at pyr_lv[i] bytes from the copies' base.  Either a pre-pass launch
    // for the small levels, copies in the workspace at pyr_off; or (gather_in_coarse) extra
    // workgroups of the coarse launch for levels between the coarse block and the finest
    // level, copies in the caller's F (written only by the finest level, which reads I and
    // alpha at full resolution), while the coarse block reads its own levels from full
    // resolution.
    int ng = 0;
    bool copy[kMaxLevels] = {};
    bool gather_in_coarse = false;
    // Single image: tile levels [pyr_first, pyr_last] run as one pyramid launch (-1: none).
    int pyr_first = -1, pyr_last = -1;
    size_t pyr_off = 0;
    size_t pyr_lv[kMaxLevels] = {};
};

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte (a null or empty range never
// does).
inline bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

// The output rule of every estimation entry point: F and B (3 planes of W*H elements of `elem`
// bytes each) share no byte with each other, with I (3 planes), alpha (1 plane) or the workspace.
inline bool outputs_alias(const void *I, const void *A, const void *F, const void *B, int W, int H,
                          int elem, const void *ws, size_t ws_bytes) {
    const size_t plane = static_cast<size_t>(W) * H * elem;
    const void *in[3] = {I, A, ws};
    const size_t in_n[3] = {3 * plane, plane, ws_bytes};
    for (int k = 0; k < 3; ++k)
        if (overlaps(F, 3 * plane, in[k], in_n[k]) || overlaps(B, 3 * plane, in[k], in_n[k]))
            return true;
    return overlaps(F, 3 * plane, B, 3 * plane);
}

int num_levels(int W, int H);
int level_size(int full, int level, int n);
bool params_valid(const fge_params &p);
// How the plan will be run.  kPlanSingle (fge_estimate_foreground): the coarse launch carries the
// gather of every intermediate level, with the copies in F, and a run of tile levels may be one
// pyramid launch.  kPlanBatched (batched and served images, whose coarse blocks run one
// workgroup per image): a gather pre-pass copies the small levels into the workspace.
enum PlanUse { kPlanBatched = 0, kPlanSingle = 1 };
fge_status make_plan(int W, int H, const fge_params &p, Plan *out, PlanUse use = kPlanBatched);

// Kernel launchers (fge_kernels.hip).  All enqueue on `stream` and return a HIP error code.
struct LevelIO {
    const void *I;      // input image, 3 planes of W*H (full resolution or a compact level copy)
    const void *A;      // alpha, W*H
    int W, H;
    const void *Fp;     // previous level F (3 planes wp*hp), nullptr: the 1x1 zero start
    const void *Bp;     // previous level B; always Fp + 3 planes (one workspace buffer)
    int wp, hp;
    void *Fo;           // this level's F, B (3 planes w*h each)
    void *Bo;
    int w, h;
    float omega, eps;
};

// Per-level source of I and alpha for the coarse kernel: the compact copy or full resolution.
struct LevelSrc {
    const void *I[kMaxLevels];
    const void *A[kMaxLevels];
    int W[kMaxLevels], H[kMaxLevels];
};

// Where an image's level data lives, given its plan, its workspace `ws` (plan.ws_bytes bytes) and
// the caller's full-resolution I, alpha, F, B.  Host-only address arithmetic.
//   level_state:  F and B of level j (the caller's buffers for the last level, else the level's
//                 ping-pong workspace buffer: F's 3 planes, then B's).
//   level_source: I and alpha of level j (its compact gather copy, else full resolution) with
//                 the size they are stored at.
//   level_io:     the record of fine level j > 0 (source, previous state, output state).
//   coarse_src:   level_source of every coarse level.
void level_state(const Plan &pl, char *ws, int j, void *F, void *B, void **f, void **b);
// Base of the compact input copies: the caller's F (gather_in_coarse) or the workspace.
char *pyr_base(const Plan &pl, char *ws, void *F);
void level_source(const Plan &pl, const char *ws, const void *F, int j, const void *I, const void *A,
                  const void **Ij, const void **Aj, int *Wj, int *Hj);
LevelIO level_io(const Plan &pl, char *ws, int j, const void *I, const void *A, void *F, void *B,
                 float omega, float eps);
LevelSrc coarse_src(const Plan &pl, const char *ws, const void *F, const void *I, const void *A);

int launch_gather(const Plan &plan, const void *I, const void *A, void *pyr, int storage,
                  void *stream);
// Whether every region of a pyramid run over levels [first, last] fits the tile kernel's LDS
// buffer (checked for every output tile), and the run's launch.
bool pyramid_fits(const Plan &plan, int first, int last);
int launch_pyramid(const Plan &plan, char *ws, const void *I, const void *A, void *F, void *B,
                   float omega, float eps, int storage, void *stream);
// The coarse block plus the gather of the staged levels in one launch (gather_in_coarse).
int launch_coarse_gather(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                         float eps, const void *I, const void *A, void *pyr, int storage,
                         void *stream);
int launch_coarse(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                  float eps, int storage, void *stream);
int launch_fine_fused(const LevelIO &io, int strip_rows, int storage, void *stream);
int launch_fine_tile(const LevelIO &io, int storage, void *stream);
// A pass of the convergence form (float32 state; the tile kernel when `tile`, else the streaming
// kernel) that also reduces the energy of the state it starts from -- the previous pass's result,
// or the previous level as the resize leaves it -- into pass_energy_parts() partial sums at epart
// (5 doubles each, fge_energy's layout; energy_final_kernel totals them).
// A non-null `skip` holding a non-zero value turns the pass into a no-op (see PassCtl).
int pass_energy_parts(const LevelIO &io, int strip_rows, bool tile);
// jacobi: the pass's two sweeps in the Jacobi order (always on the tile kernel).
int launch_pass_energy(const LevelIO &io, int strip_rows, bool tile, double *epart,
                       const int *skip, void *stream, bool jacobi = false);
int launch_naive_level(const LevelIO &io, int iters, int storage, void *stream);


// ---- kernel argument records (shared by host and device code) ---------------------------

// Coarse block of one image: levels [0, nc) in one workgroup.
struct CoarseArgs {
    LevelSrc src;       // per level: I, alpha and their size (compact copy or full resolution)
    void *Fo;
    void *Bo;
    int nc;
    int lw[kMaxLevels], lh[kMaxLevels], lit[kMaxLevels];
    float omega, eps;
};

// One fine level on the LDS tile kernel: 32x32 output tiles, tiles_x per row.
struct TileArgs {
    const void *I;
    const void *A;
    int W, H;
    const void *Fp;
    const void *Bp;
    int wp, hp;
    void *Fo;
    void *Bo;
    int w, h;
    int tiles_x;
    float omega, eps;
};

// A run of consecutive tile levels in one launch (pyramid kernel): per level its I and alpha
// source and its size; the stored level before the run; the run's last level's outputs.
constexpr int kPyrMaxLevels = 8;
struct PyramidLevel {
    const void *I;
    const void *A;
    int W, H;
    int w, h;
};
struct PyramidArgs {
    int nl;
    PyramidLevel lv[kPyrMaxLevels];
    const void *Fp;
    const void *Bp;
    int wp, hp;
    void *Fo;
    void *Bo;
    int tiles_x, tiles;
    float omega, eps;
};

// One fine level on the streaming kernel: nx x ny strips of strip_rows rows.
struct FineArgs {
    const void *I;
    const void *A;
    int W, H;
    const void *Fp;
    const void *Bp;
    int wp, hp;
    void *Fo;
    void *Bo;
    int w, h;
    float omega, eps;
    int nx, ny, strip_rows;
};

// Gather pre-pass of one image: compact copies of levels [0, ng).
struct GatherArgs {
    const void *I;
    const void *A;
    int W, H;
    char *pyr;
    int ng;
    int lw[kMaxLevels], lh[kMaxLevels];
    long long first[kMaxLevels + 1];   // first concatenated pixel of each level
    long long off[kMaxLevels];         // byte offset of each level's planes in pyr
};

// One unit of work of a batched launch: a strip or tile of descriptor `desc`.
struct WorkItem {
    int desc;   // index into the launch's descriptor table
    int unit;   // strip (streaming) or tile index
};

// Descriptor builders (host side; geometry as the single-image launches use it).
void make_fine_args(const LevelIO &io, int strip_rows, FineArgs *a);
void make_tile_args(const LevelIO &io, TileArgs *a);
int fine_units(const FineArgs &a);
// Strip height for one batched streaming launch over levels of sizes w[k] x h[k]; 0 = none
// fits (too little work in the launch: each level takes its own automatic height).
int launch_strip_rows(const int *w, const int *h, int n);
int tile_units(const TileArgs &a);
void make_coarse_args(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                      float eps, CoarseArgs *a);
void make_gather_args(const Plan &plan, const void *I, const void *A, void *pyr, GatherArgs *a);
long long gather_units(const GatherArgs &a);

// Energy of (F, B) (w x h, element type state_storage) against I, alpha (W x H, element type
// storage, read through the level's nearest map) into out[0..5] (fge_energy's layout); `part`
// holds energy_blocks(w, h) * 5 doubles.  A non-null `stop` holding a non-zero value makes both
// launches no-ops.
int energy_blocks(int w, int h);
int launch_energy(const void *I, const void *A, int W, int H, const void *F, const void *B, int w,
                  int h, float omega, float eps, int storage, int state_storage, const int *stop,
                  double *part, double *out, void *stream);
// The same with F and B of size fw x fh read through the nearest map onto the w x h level (the
// energy of a level's start state: the previous level's result as the resize leaves it).
int launch_energy_mapped(const void *I, const void *A, int W, int H, const void *F, const void *B,
                         int fw, int fh, int w, int h, float omega, float eps, int storage,
                         int state_storage, const int *stop, double *part, double *out,
                         void *stream);
// Totals nb partial sums of fge_energy's layout (5 doubles each) into out[0..5], as fge_energy
// reports them (out[0] the energy).
int launch_energy_final(const double *part, int nb, double *out, void *stream);
// launch_energy's partial sums, then in one launch their total and the stop rule of the level
// loop tested after every sweep (k = 0: the level's resized start; k > 0 records count = k and
// sets stop when |eprev - E| <= tol eprev or k >= kmax; eprev = E).  Both launches are no-ops
// once stop is set.
int launch_energy_check(const void *I, const void *A, int W, int H, const void *F, const void *B,
                        int w, int h, float omega, float eps, int storage, int state_storage,
                        double *part, double *out, double *eprev, int *stop, int *count,
                        double tol, int k, int kmax, void *stream);
// The convergence form's stop rule on the device, beside the host's: pass m's total (the energy
// after pass m - 1) also updates ctl -- m == 1 starts the level (e_prev = that energy, stop = 0);
// m > 1 sets stop when |e_prev - e| <= tol e_prev, else e_prev = e.  Once stop is set the later
// passes and totals of the level do nothing (the host, judging the same values, stops there too).
struct PassCtl {
    double e_prev;
    int stop;
    int pad;
};
// out: 7 doubles of host-visible memory -- the total as fge_energy's 6 outputs, then seq, written
// last (behind a system-scope fence) so that the host can poll for it.
int launch_pass_final(const double *part, int nb, double *out, PassCtl *ctl, int m, double tol,
                      long seq, void *stream);

// Level loop with the convergence stop or the Jacobi order (fge_converge.hip); tol < 0 runs the
// fixed counts.
size_t converge_workspace_bytes(int W, int H, const fge_params &p);
fge_status estimate_converge(const void *I, const void *A, int W, int H, const fge_params &p,
                             double tol, int max_sweeps, void *F, void *B, int32_t *sweeps_out,
                             void *workspace, size_t workspace_bytes, void *stream);

// The convergence form in passes of two sweeps on the fused kernels (fge_converge.hip); smooth:
// with the smooth resize variant (area copies of I and alpha, the previous level's F and B resized
// bilinearly before the first pass; no coarse block).
size_t converge_passes_workspace_bytes(int W, int H, const fge_params &p, bool smooth = false);
fge_status estimate_converge_passes(const void *I, const void *A, int W, int H,
                                    const fge_params &p, double tol, int max_passes, void *F,
                                    void *B, int32_t *passes_out, void *workspace,
                                    size_t workspace_bytes, void *stream, bool smooth = false);

// Batched launches: descriptor tables, work lists and counters are device pointers.  Every
// batched tile or streaming launch uses kQueueCounters counters (one work queue per XCD).
constexpr int kQueueCounters = 8;
int launch_zero(int *d, int n, void *stream);
int launch_gather_batch(const GatherArgs *descs, const long long *first, int n, long long total,
                        int storage, void *stream);
int launch_coarse_batch(const CoarseArgs *descs, int n, int storage, void *stream);
// Coarse levels [0, a.nc) in the convergence form, one workgroup, float32 inputs and state: a
// level runs passes of two sweeps until a pass changes its energy by at most tol times the value
// before it, or max_passes passes; the passes of level l go to counts[l] (device-visible memory).
int launch_coarse_converge(const CoarseArgs &a, double tol, int max_passes, int *counts,
                           void *stream);
int launch_fine_batch(const FineArgs *descs, const WorkItem *items, int nitems, int *counter,
                      int storage, void *stream);
int launch_tile_batch(const TileArgs *descs, const WorkItem *items, int nitems, int *counter,
                      int storage, void *stream);

}  // namespace fge
