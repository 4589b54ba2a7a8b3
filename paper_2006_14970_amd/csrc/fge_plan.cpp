// Level planner: Algorithm 1's schedule (level count, level sizes, sweeps per level) and the
// workspace layout of the device path.  Host-only code.
#include <cmath>
#include <cstring>

#include "fge_internal.h"

namespace fge {

// Algorithm 1: n_l = ceil(log2(max(W, H))); a 1x1 input still runs one level.
int num_levels(int W, int H) {
    const int m = W > H ? W : H;
    int n = 0;
    while ((1 << n) < m) ++n;
    return n < 1 ? 1 : n;
}

// Algorithm 1: round(full^(level / n)).  For full <= 32767 and n <= 15 the value is never
// closer than ~1e-9 (relative) to a half-integer, far above double rounding error, so the
// double evaluation is exact (checked exhaustively against exact integer arithmetic in tests).
int level_size(int full, int level, int n) {
    const double v = std::pow(static_cast<double>(full), static_cast<double>(level) / n);
    return static_cast<int>(std::lround(v));
}

bool params_valid(const fge_params &p) {
    if (p.size != sizeof(fge_params)) return false;
    if (!(p.omega >= 0.0f) || !std::isfinite(p.omega)) return false;
    if (!(p.eps_r > 0.0f) || !std::isfinite(p.eps_r)) return false;   // eps_r > 0 keeps det > 0
    if (p.small_size < 0 || p.iters_small < 0 || p.iters_big < 0) return false;
    if (p.iters_small > 1000 || p.iters_big > 1000) return false;
    if (p.storage != FGE_F32 && p.storage != FGE_F16) return false;
    if (p.order != FGE_REDBLACK && p.order != FGE_JACOBI) return false;
    if (p.kernel < FGE_KERNEL_AUTO || p.kernel > FGE_KERNEL_NAIVE) return false;
    if (p.strip_rows < 0 || p.strip_rows > 1 << 20) return false;
    if (p.coarse_max_px < -1 || p.coarse_max_px > kCoarseMaxPx) return false;
    if (p.tile_max_px < -1) return false;
    return true;
}

static size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

fge_status make_plan(int W, int H, const fge_params &p, Plan *out, PlanUse use) {
    if (W < 1 || H < 1 || W > kMaxSide || H > kMaxSide) return FGE_EINVAL;
    if (!params_valid(p)) return FGE_EINVAL;
    Plan pl;
    pl.W = W;
    pl.H = H;
    pl.n = num_levels(W, H);
    pl.elem = p.storage == FGE_F16 ? 2 : 4;
    for (int i = 0; i < pl.n; ++i) {
        const int w = level_size(W, i + 1, pl.n);
        const int h = level_size(H, i + 1, pl.n);
        const bool small = w <= p.small_size && h <= p.small_size;
        pl.lv[i] = {w, h, small ? p.iters_small : p.iters_big};
    }
    // The coarse block and the fused fine kernels sweep in red-black order; the Jacobi order
    // runs every level on per-level kernels.
    const bool jacobi = p.order == FGE_JACOBI;
    if (jacobi && p.kernel == FGE_KERNEL_FUSED) return FGE_EUNSUPPORTED;
    // Coarse block: the longest prefix of levels with w*h <= limit (sizes grow with l).  The
    // automatic limit keeps the block to the levels up to 1024 px -- larger ones run faster on
    // the tile kernel, spread over several workgroups -- plus every level whose sweep count is
    // not 2, which only the block or the per-level kernels can run (low-resolution levels when
    // small_size exceeds 32).
    const bool auto_limit = p.coarse_max_px == 0;
    const int limit = jacobi ? -1 : (auto_limit ? kCoarseAutoPx : p.coarse_max_px);
    pl.nc = 0;
    // A coarse level must also fit the block's LDS (kCoarseMaxPx pixels) and have at most
    // kCoarseMaxPairs pairs of columns (thin levels of odd width can exceed that while still
    // having <= 4096 pixels).
    if (limit > 0)
        while (pl.nc < pl.n) {
            const long px = static_cast<long>(pl.lv[pl.nc].w) * pl.lv[pl.nc].h;
            const bool fits = px <= kCoarseMaxPx &&
                              static_cast<long>((pl.lv[pl.nc].w + 1) / 2) * pl.lv[pl.nc].h <= kCoarseMaxPairs;
            const bool wanted = px <= limit || (auto_limit && pl.lv[pl.nc].iters != 2);
            if (!fits || !wanted) break;
            ++pl.nc;
        }
    // Fine levels: the fused kernels (tile and streaming) implement exactly two sweeps per
    // level and need a previous level; mid-size levels take the tile kernel, large ones the
    // streaming kernel.
    const long tile_max = p.tile_max_px == 0 ? kTileMaxPxDefault : p.tile_max_px;
    for (int i = 0; i < pl.n; ++i) pl.kind[i] = kKindCoarse;
    for (int i = pl.nc; i < pl.n; ++i) {
        const bool can_fuse = pl.lv[i].iters == 2 && i > 0;
        if (p.kernel == FGE_KERNEL_FUSED && !can_fuse) return FGE_EUNSUPPORTED;
        if (p.kernel == FGE_KERNEL_NAIVE || jacobi || !can_fuse)
            pl.kind[i] = kKindNaive;
        else if (static_cast<long>(pl.lv[i].w) * pl.lv[i].h <= tile_max ||
                 3 * static_cast<long long>(W) * H * pl.elem >= (1LL << 32))
            pl.kind[i] = kKindTile;   // the streaming kernel addresses each tensor in 4 GiB
        else
            pl.kind[i] = kKindStream;
    }
    // Compact inputs.  A level below full resolution reads I and alpha through the nearest map,
    // which touches far more cache lines than it uses (all of every mapped row at 2:1, one line
    // per pixel further down).  Not when the full image is itself small.
    //  - Single image with a coarse block: the coarse block runs on one CU for tens of
    //    microseconds while the rest of the GPU idles, so the same launch copies the inputs of
    //    every level after the block except the finest into compact planes, and the coarse
    //    block reads its own (tiny) levels from full resolution.  The staged levels then read
    //    their inputs with the identity map (the streaming kernel's paired loads apply to 2:1
    //    levels).  The copies live in F, which only the finest level writes.
    //  - Otherwise a pre-pass launch copies the small coarse and tile levels.
    pl.ng = 0;
    pl.gather_in_coarse = false;
    for (int i = 0; i < pl.n; ++i) pl.copy[i] = false;
    if (static_cast<long>(W) * H > kGatherMaxPx) {
        size_t staged = 0;   // bytes of the staged copies, which must fit in F (3 W H elements)
        for (int i = pl.nc; i < pl.n - 1; ++i)
            staged += align256(4 * static_cast<size_t>(pl.lv[i].w) * pl.lv[i].h * pl.elem);
        if (use == kPlanSingle && pl.nc > 0 && pl.n - 1 > pl.nc && p.kernel != FGE_KERNEL_NAIVE &&
            staged <= 3 * static_cast<size_t>(W) * H * pl.elem) {
            pl.gather_in_coarse = true;
            for (int i = pl.nc; i < pl.n - 1; ++i) pl.copy[i] = true;
        } else {
            for (int i = 0; i < pl.n && (pl.kind[i] == kKindCoarse || pl.kind[i] == kKindTile) &&
                            static_cast<long>(pl.lv[i].w) * pl.lv[i].h <= kGatherMaxPx;
                 ++i)
                pl.copy[i] = true;
        }
        for (int i = 0; i < pl.n; ++i) pl.ng += pl.copy[i];
        if (pl.ng == 0) pl.gather_in_coarse = false;
    }
    // Single image: a run of at least two tile levels becomes one pyramid launch, when every
    // region it needs fits the tile buffer.  The run stops before the finest level when the
    // staged copies live in F: the finest level's stores would overwrite copies that other
    // workgroups of the same launch still read.
    pl.pyr_first = pl.pyr_last = -1;
    if (use == kPlanSingle && p.kernel != FGE_KERNEL_NAIVE) {
        int a = pl.nc;
        while (a < pl.n && pl.kind[a] != kKindTile) ++a;
        int b = a;
        while (b + 1 < pl.n && pl.kind[b + 1] == kKindTile && b + 1 - a + 1 <= kPyrMaxLevels) ++b;
        if (pl.gather_in_coarse && b == pl.n - 1) --b;
        if (a < pl.n && b > a && pyramid_fits(pl, a, b)) {
            pl.pyr_first = a;
            pl.pyr_last = b;
        }
    }
    // Workspace: the state of every stored level except the last goes through one of two
    // buffers, alternating from the last level down, so a level never writes the buffer its
    // input is in.  Stored are the levels from nc-1 on (coarser ones live in LDS) except those
    // inside a pyramid run, which stay in LDS too.
    const int first_mat = pl.nc > 0 ? pl.nc - 1 : 0;
    for (int i = 0; i < pl.n; ++i) pl.buf_of[i] = -1;
    for (int i = pl.n - 2, k = 0; i >= first_mat; --i) {
        if (i >= pl.pyr_first && i < pl.pyr_last) continue;
        const int b = k++ & 1;
        pl.buf_of[i] = b;
        const size_t px = static_cast<size_t>(pl.lv[i].w) * pl.lv[i].h;
        if (px > pl.buf_px[b]) pl.buf_px[b] = px;
    }
    pl.buf_off[0] = 0;
    pl.buf_off[1] = align256(6 * pl.buf_px[0] * pl.elem);
    pl.ws_bytes = pl.buf_px[1] ? pl.buf_off[1] + align256(6 * pl.buf_px[1] * pl.elem)
                               : (pl.buf_px[0] ? pl.buf_off[1] : 0);
    pl.pyr_off = pl.ws_bytes;
    size_t pyr = 0;
    for (int i = 0; i < pl.n; ++i) {
        if (!pl.copy[i]) continue;
        pl.pyr_lv[i] = pyr;
        pyr += align256(4 * static_cast<size_t>(pl.lv[i].w) * pl.lv[i].h * pl.elem);
    }
    if (!pl.gather_in_coarse) pl.ws_bytes += pyr;
    *out = pl;
    return FGE_OK;
}

void level_state(const Plan &pl, char *ws, int j, void *F, void *B, void **f, void **b) {
    if (j == pl.n - 1) {
        *f = F;
        *b = B;
        return;
    }
    if (pl.buf_of[j] < 0) {   // not stored (inside the coarse block or a pyramid run)
        *f = *b = nullptr;
        return;
    }
    char *base = ws + pl.buf_off[pl.buf_of[j]];
    *f = base;
    *b = base + 3 * static_cast<size_t>(pl.lv[j].w) * pl.lv[j].h * pl.elem;
}

char *pyr_base(const Plan &pl, char *ws, void *F) {
    return pl.gather_in_coarse ? static_cast<char *>(F) : ws + pl.pyr_off;
}

void level_source(const Plan &pl, const char *ws, const void *F, int j, const void *I, const void *A,
                  const void **Ij, const void **Aj, int *Wj, int *Hj) {
    if (pl.copy[j]) {
        const char *base = pyr_base(pl, const_cast<char *>(ws), const_cast<void *>(F)) + pl.pyr_lv[j];
        *Ij = base;
        *Aj = base + 3 * static_cast<size_t>(pl.lv[j].w) * pl.lv[j].h * pl.elem;
        *Wj = pl.lv[j].w;
        *Hj = pl.lv[j].h;
    } else {
        *Ij = I;
        *Aj = A;
        *Wj = pl.W;
        *Hj = pl.H;
    }
}

LevelIO level_io(const Plan &pl, char *ws, int j, const void *I, const void *A, void *F, void *B,
                 float omega, float eps) {
    LevelIO io{};
    level_source(pl, ws, F, j, I, A, &io.I, &io.A, &io.W, &io.H);
    if (j > 0) {
        void *fp, *bp;
        level_state(pl, ws, j - 1, F, B, &fp, &bp);
        io.Fp = fp;
        io.Bp = bp;
        io.wp = pl.lv[j - 1].w;
        io.hp = pl.lv[j - 1].h;
    } else {
        io.Fp = io.Bp = nullptr;
        io.wp = io.hp = 1;
    }
    level_state(pl, ws, j, F, B, &io.Fo, &io.Bo);
    io.w = pl.lv[j].w;
    io.h = pl.lv[j].h;
    io.omega = omega;
    io.eps = eps;
    return io;
}

LevelSrc coarse_src(const Plan &pl, const char *ws, const void *F, const void *I, const void *A) {
    LevelSrc src{};
    for (int j = 0; j < pl.nc; ++j)
        level_source(pl, ws, F, j, I, A, &src.I[j], &src.A[j], &src.W[j], &src.H[j]);
    return src;
}

}  // namespace fge
