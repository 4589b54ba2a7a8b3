// Internal declarations shared by the planner, the kernels and the C ABI of libfge.
#pragma once

#include <cstddef>
#include <cstdint>

#include "fge.h"

namespace fge {

constexpr int kMaxLevels = 16;         // 32767 needs 15 levels
constexpr int kMaxSide = 32767;        // keeps x * w_src inside int32
constexpr int kCoarseMaxPx = 4096;     // LDS-resident coarse levels: 2 float4 per pixel = 128 KB
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
    // of one level at that level's size.  Level i < n-1 lives in buffer (n - 2 - i) % 2; the
    // last level is written straight into the caller's F and B.
    size_t buf_off[2] = {0, 0};
    size_t buf_px[2] = {0, 0};
    size_t ws_bytes = 0;
    int kind[kMaxLevels] = {};     // per fine level: a LevelKind
    // Gather pre-pass: levels [0, ng) get a compact copy of their resized I (3 planes) and alpha
    // (1 plane) at pyr_off + pyr_lv[i] bytes of the workspace.
    int ng = 0;
    size_t pyr_off = 0;
    size_t pyr_lv[kMaxLevels] = {};
};

int num_levels(int W, int H);
int level_size(int full, int level, int n);
bool params_valid(const fge_params &p);
fge_status make_plan(int W, int H, const fge_params &p, Plan *out);

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

int launch_gather(const Plan &plan, const void *I, const void *A, void *pyr, int storage,
                  void *stream);
int launch_coarse(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                  float eps, int storage, void *stream);
int launch_fine_fused(const LevelIO &io, int strip_rows, int storage, void *stream);
int launch_fine_tile(const LevelIO &io, int storage, void *stream);
int launch_naive_level(const LevelIO &io, int iters, int storage, void *stream);

}  // namespace fge
