// Batched estimation of images of different sizes (C ABI in include/fge.h).
//
// Every image follows its own level plan (Algorithm 1), exactly as fge_estimate_foreground runs
// it, so a batched image's F and B are bit-identical to its single-image result.  The levels of
// all images are aligned from the finest: at fine step s (0 <= s < S) image i runs its level
// n_i - S + s when that level is above its coarse block.  One run is:
//   1. one async upload of the descriptor tables and work lists (pinned staging -> workspace),
//   2. a fill kernel zeroing the per-launch work counters,
//   3. the batched gather pre-pass (compact inputs of every image's small levels),
//   4. the batched coarse block (one workgroup per image),
//   5. per fine step, one persistent tile-kernel launch and one persistent streaming-kernel
//      launch, whose waves pull (descriptor, strip|tile) items from the step's counter.
// The sequence can be captured once into a hipGraph and replayed with the same pointers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "fge_internal.h"

namespace {

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

struct Launch {
    int kind;            // fge::kKindTile or fge::kKindStream
    int step;
    std::vector<std::pair<int, int>> lv;   // (image, level)
    size_t desc_off = 0, item_off = 0;     // byte offsets in the table region
    int nitems = 0;
    int counter = 0;
    int rows = 0;        // streaming strip height (0: each level's automatic height)
};

}  // namespace

struct fge_batch {
    int n = 0;
    fge_params prm{};
    std::vector<fge::Plan> plans;
    std::vector<size_t> img_off;            // per image region in the workspace
    int S = 0;                              // fine steps
    std::vector<Launch> launches;           // in execution order
    // table region (after the images' regions)
    size_t tab_off = 0, tab_bytes = 0;
    size_t gather_desc_off = 0, gather_first_off = 0, coarse_desc_off = 0;
    std::vector<int> gather_imgs, coarse_imgs;
    long long gather_total = 0;
    size_t cnt_off = 0;
    int ncnt = 0;
    size_t ws_bytes = 0;
    // staging
    char *staging = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char *graph_staging = nullptr;
    // Recorded after every replay: the graph's upload node reads graph_staging when it runs, so
    // a new capture (which refills graph_staging) and destroy wait for it first.
    hipEvent_t replayed = nullptr;
    bool replay_pending = false;
};

namespace {

fge::LevelIO level_io(const fge_batch &b, int i, int j, char *ws, const void *const *I,
                      const void *const *A, void *const *F, void *const *B) {
    return fge::level_io(b.plans[i], ws + b.img_off[i], j, I[i], A[i], F[i], B[i], b.prm.omega,
                         b.prm.eps_r);
}

// Fill the table region image (descriptors and work lists) for these pointers.
void fill_tables(const fge_batch &b, char *tab, char *ws, const void *const *I,
                 const void *const *A, void *const *F, void *const *B) {
    std::memset(tab, 0, b.tab_bytes);
    auto *gd = reinterpret_cast<fge::GatherArgs *>(tab + b.gather_desc_off);
    auto *gf = reinterpret_cast<long long *>(tab + b.gather_first_off);
    long long first = 0;
    for (size_t k = 0; k < b.gather_imgs.size(); ++k) {
        const int i = b.gather_imgs[k];
        fge::make_gather_args(b.plans[i], I[i], A[i], ws + b.img_off[i] + b.plans[i].pyr_off, &gd[k]);
        gf[k] = first;
        first += fge::gather_units(gd[k]);
    }
    auto *cd = reinterpret_cast<fge::CoarseArgs *>(tab + b.coarse_desc_off);
    for (size_t k = 0; k < b.coarse_imgs.size(); ++k) {
        const int i = b.coarse_imgs[k];
        const fge::Plan &pl = b.plans[i];
        char *iws = ws + b.img_off[i];
        const fge::LevelSrc src = fge::coarse_src(pl, iws, F[i], I[i], A[i]);
        void *fo, *bo;
        fge::level_state(pl, iws, pl.nc - 1, F[i], B[i], &fo, &bo);
        fge::make_coarse_args(pl, src, fo, bo, b.prm.omega, b.prm.eps_r, &cd[k]);
    }
    for (const Launch &L : b.launches) {
        auto *items = reinterpret_cast<fge::WorkItem *>(tab + L.item_off);
        int m = 0;
        for (size_t d = 0; d < L.lv.size(); ++d) {
            const fge::LevelIO io = level_io(b, L.lv[d].first, L.lv[d].second, ws, I, A, F, B);
            int units;
            if (L.kind == fge::kKindTile) {
                auto *td = reinterpret_cast<fge::TileArgs *>(tab + L.desc_off);
                fge::make_tile_args(io, &td[d]);
                units = fge::tile_units(td[d]);
            } else {
                auto *fd = reinterpret_cast<fge::FineArgs *>(tab + L.desc_off);
                fge::make_fine_args(io, L.rows, &fd[d]);
                units = fge::fine_units(fd[d]);
            }
            for (int u = 0; u < units; ++u) items[m++] = fge::WorkItem{static_cast<int>(d), u};
        }
    }
}

fge_status enqueue(fge_batch &b, const void *const *I, const void *const *A, void *const *F,
                   void *const *B, void *workspace, hipStream_t s, char *staging, bool capture) {
    char *ws = static_cast<char *>(workspace);
    fill_tables(b, staging, ws, I, A, F, B);
    if (hipMemcpyAsync(ws + b.tab_off, staging, b.tab_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return FGE_EHIP;
    if (!capture) {
        if (hipEventRecord(b.staged, s) != hipSuccess) return FGE_EHIP;
        b.staged_pending = true;
    }
    int *cnt = reinterpret_cast<int *>(ws + b.cnt_off);
    if (fge::launch_zero(cnt, b.ncnt, s)) return FGE_EHIP;
    const int st = b.prm.storage;
    char *tab = ws + b.tab_off;
    if (!b.gather_imgs.empty() &&
        fge::launch_gather_batch(reinterpret_cast<const fge::GatherArgs *>(tab + b.gather_desc_off),
                                 reinterpret_cast<const long long *>(tab + b.gather_first_off),
                                 static_cast<int>(b.gather_imgs.size()), b.gather_total, st, s))
        return FGE_EHIP;
    if (!b.coarse_imgs.empty() &&
        fge::launch_coarse_batch(reinterpret_cast<const fge::CoarseArgs *>(tab + b.coarse_desc_off),
                                 static_cast<int>(b.coarse_imgs.size()), st, s))
        return FGE_EHIP;
    for (const Launch &L : b.launches) {
        int err;
        if (L.kind == fge::kKindTile)
            err = fge::launch_tile_batch(reinterpret_cast<const fge::TileArgs *>(tab + L.desc_off),
                                         reinterpret_cast<const fge::WorkItem *>(tab + L.item_off),
                                         L.nitems, cnt + L.counter, st, s);
        else
            err = fge::launch_fine_batch(reinterpret_cast<const fge::FineArgs *>(tab + L.desc_off),
                                         reinterpret_cast<const fge::WorkItem *>(tab + L.item_off),
                                         L.nitems, cnt + L.counter, st, s);
        if (err) return FGE_EHIP;
    }
    return FGE_OK;
}

fge_status check_ptrs(const fge_batch &b, const void *const *I, const void *const *A,
                      void *const *F, void *const *B, const void *workspace, size_t bytes) {
    if (!I || !A || !F || !B) return FGE_EINVAL;
    for (int i = 0; i < b.n; ++i) {
        if (!I[i] || !A[i] || !F[i] || !B[i]) return FGE_EINVAL;
        const fge::Plan &pl = b.plans[i];
        if (fge::outputs_alias(I[i], A[i], F[i], B[i], pl.W, pl.H, pl.elem, workspace, bytes))
            return FGE_EINVAL;
    }
    if (!workspace || bytes < b.ws_bytes) return FGE_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return FGE_EWORKSPACE;
    return FGE_OK;
}

}  // namespace

extern "C" {

fge_status fge_batch_create(int32_t n, const int32_t *H, const int32_t *W, const fge_params *p,
                            fge_batch **out) {
    if (!out || n < 1 || n > (1 << 16) || !W || !H) return FGE_EINVAL;
    *out = nullptr;
    fge_params prm;
    if (p) prm = *p; else fge_default_params(&prm);
    fge_batch *b = new (std::nothrow) fge_batch();
    if (!b) return FGE_ENOMEM;
    b->n = n;
    b->prm = prm;
    b->plans.resize(n);
    b->img_off.resize(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const fge_status st = fge::make_plan(W[i], H[i], prm, &b->plans[i]);
        if (st != FGE_OK) {
            delete b;
            return st;
        }
        const fge::Plan &pl = b->plans[i];
        // the batched path needs the coarse block for the first level and fused fine levels
        if (pl.nc < 1) {
            delete b;
            return FGE_EUNSUPPORTED;
        }
        for (int j = pl.nc; j < pl.n; ++j)
            if (pl.kind[j] != fge::kKindTile && pl.kind[j] != fge::kKindStream) {
                delete b;
                return FGE_EUNSUPPORTED;
            }
        b->img_off[i] = off;
        off += align256(pl.ws_bytes);
        b->S = std::max(b->S, pl.n - pl.nc);
    }
    // Fine steps aligned from the finest level; per step a tile launch and a streaming launch,
    // their levels ordered largest first so the long items start first.
    for (int s = 0; s < b->S; ++s) {
        for (int kind : {fge::kKindTile, fge::kKindStream}) {
            Launch L;
            L.kind = kind;
            L.step = s;
            for (int i = 0; i < n; ++i) {
                const fge::Plan &pl = b->plans[i];
                const int j = pl.n - b->S + s;
                if (j >= pl.nc && j < pl.n && pl.kind[j] == kind) L.lv.push_back({i, j});
            }
            if (L.lv.empty()) continue;
            std::stable_sort(L.lv.begin(), L.lv.end(), [&](const auto &x, const auto &y) {
                const auto &a = b->plans[x.first].lv[x.second];
                const auto &c = b->plans[y.first].lv[y.second];
                return static_cast<long>(a.w) * a.h > static_cast<long>(c.w) * c.h;
            });
            b->launches.push_back(std::move(L));
        }
    }
    for (int i = 0; i < n; ++i) {
        if (b->plans[i].ng > 0) b->gather_imgs.push_back(i);
        b->coarse_imgs.push_back(i);
    }
    // Table region layout (sizes do not depend on the pointers).
    size_t t = 0;
    b->gather_desc_off = t;
    t = align256(t + b->gather_imgs.size() * sizeof(fge::GatherArgs));
    b->gather_first_off = t;
    t = align256(t + b->gather_imgs.size() * sizeof(long long));
    b->coarse_desc_off = t;
    t = align256(t + b->coarse_imgs.size() * sizeof(fge::CoarseArgs));
    for (const int i : b->gather_imgs) {
        const fge::Plan &pl = b->plans[i];
        for (int j = 0; j < pl.n; ++j)
            if (pl.copy[j]) b->gather_total += static_cast<long long>(pl.lv[j].w) * pl.lv[j].h;
    }
    int counter = 0;
    for (Launch &L : b->launches) {
        if (L.kind == fge::kKindStream) {
            if (prm.strip_rows > 0) {
                L.rows = prm.strip_rows;
            } else {
                std::vector<int> ws, hs;
                for (const auto &iv : L.lv) {
                    ws.push_back(b->plans[iv.first].lv[iv.second].w);
                    hs.push_back(b->plans[iv.first].lv[iv.second].h);
                }
                L.rows = fge::launch_strip_rows(ws.data(), hs.data(), static_cast<int>(ws.size()));
            }
        }
        L.desc_off = t;
        const size_t dsz = L.kind == fge::kKindTile ? sizeof(fge::TileArgs) : sizeof(fge::FineArgs);
        t = align256(t + L.lv.size() * dsz);
        // unit counts depend only on sizes and strip rows: compute with null pointers
        int units = 0;
        for (const auto &iv : L.lv) {
            const fge::Level &lv = b->plans[iv.first].lv[iv.second];
            fge::LevelIO io{};
            io.w = lv.w;
            io.h = lv.h;
            if (L.kind == fge::kKindTile) {
                fge::TileArgs a;
                fge::make_tile_args(io, &a);
                units += fge::tile_units(a);
            } else {
                fge::FineArgs a;
                fge::make_fine_args(io, L.rows, &a);
                units += fge::fine_units(a);
            }
        }
        L.nitems = units;
        L.item_off = t;
        t = align256(t + static_cast<size_t>(units) * sizeof(fge::WorkItem));
        L.counter = counter;
        counter += fge::kQueueCounters;
    }
    b->tab_bytes = t;
    b->tab_off = off;
    off = align256(off + t);
    b->cnt_off = off;
    b->ncnt = counter;
    off = align256(off + std::max(1, counter) * sizeof(int));
    b->ws_bytes = off;
    *out = b;   // pinned staging and the upload event are created by the first run (host-only here)
    return FGE_OK;
}

void fge_batch_destroy(fge_batch *b) {
    if (!b) return;
    if (b->replayed) {
        if (b->replay_pending) (void)hipEventSynchronize(b->replayed);
        (void)hipEventDestroy(b->replayed);
    }
    if (b->staged) {
        if (b->staged_pending) (void)hipEventSynchronize(b->staged);
        (void)hipEventDestroy(b->staged);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->staging) (void)hipHostFree(b->staging);
    if (b->graph_staging) (void)hipHostFree(b->graph_staging);
    delete b;
}

size_t fge_batch_workspace_bytes(const fge_batch *b) { return b ? b->ws_bytes : 0; }

int32_t fge_batch_steps(const fge_batch *b) { return b ? b->S : 0; }

int32_t fge_batch_launch_count(const fge_batch *b) {
    if (!b) return 0;
    return 2 + (b->gather_imgs.empty() ? 0 : 1) + (b->coarse_imgs.empty() ? 0 : 1) +
           static_cast<int32_t>(b->launches.size());
}

fge_status fge_batch_run(fge_batch *b, const void *const *I, const void *const *alpha,
                         void *const *F, void *const *B, void *workspace, size_t workspace_bytes,
                         void *stream) {
    if (!b) return FGE_EINVAL;
    const fge_status st = check_ptrs(*b, I, alpha, F, B, workspace, workspace_bytes);
    if (st != FGE_OK) return st;
    if (!b->staging &&
        (hipHostMalloc(reinterpret_cast<void **>(&b->staging), std::max<size_t>(b->tab_bytes, 256),
                       hipHostMallocDefault) != hipSuccess ||
         hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess))
        return FGE_EHIP;
    // the staging buffer is reused: wait until the previous run's upload has been executed
    if (b->staged_pending) {
        if (hipEventSynchronize(b->staged) != hipSuccess) return FGE_EHIP;
        b->staged_pending = false;
    }
    return enqueue(*b, I, alpha, F, B, workspace, static_cast<hipStream_t>(stream), b->staging, false);
}

fge_status fge_batch_capture(fge_batch *b, const void *const *I, const void *const *alpha,
                             void *const *F, void *const *B, void *workspace,
                             size_t workspace_bytes, void *stream) {
    if (!b || !stream) return FGE_EINVAL;
    const fge_status st = check_ptrs(*b, I, alpha, F, B, workspace, workspace_bytes);
    if (st != FGE_OK) return st;
    // Replays of the previous graph may still be queued: their upload node reads graph_staging,
    // which this capture refills.
    if (b->replay_pending) {
        if (hipEventSynchronize(b->replayed) != hipSuccess) return FGE_EHIP;
        b->replay_pending = false;
    }
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (!b->graph_staging &&
        hipHostMalloc(reinterpret_cast<void **>(&b->graph_staging), std::max<size_t>(b->tab_bytes, 256),
                      hipHostMallocDefault) != hipSuccess)
        return FGE_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return FGE_EHIP;
    const fge_status est = enqueue(*b, I, alpha, F, B, workspace, s, b->graph_staging, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (est != FGE_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return est != FGE_OK ? est : FGE_EHIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return FGE_EHIP;
    return FGE_OK;
}

fge_status fge_batch_replay(fge_batch *b, void *stream) {
    if (!b || !b->exec) return FGE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!b->replayed && hipEventCreateWithFlags(&b->replayed, hipEventDisableTiming) != hipSuccess)
        return FGE_EHIP;
    // Replays share the workspace and its counters, so each one waits for the previous one
    // (possibly on another stream); the event of the last replay then covers them all.
    if (b->replay_pending && hipStreamWaitEvent(s, b->replayed, 0) != hipSuccess) return FGE_EHIP;
    if (hipGraphLaunch(b->exec, s) != hipSuccess) return FGE_EHIP;
    if (hipEventRecord(b->replayed, s) != hipSuccess) return FGE_EHIP;
    b->replay_pending = true;
    return FGE_OK;
}

size_t fge_batch_workspace_bytes_for(int32_t n, const int32_t *H, const int32_t *W,
                                     const fge_params *p) {
    fge_batch *b = nullptr;
    if (fge_batch_create(n, H, W, p, &b) != FGE_OK) return 0;
    const size_t v = b->ws_bytes;
    fge_batch_destroy(b);
    return v;
}

fge_status fge_estimate_foreground_batch(int32_t n, const void *const *I, const void *const *alpha,
                                         const int32_t *H, const int32_t *W, const fge_params *p,
                                         void *const *F, void *const *B, void *workspace,
                                         size_t workspace_bytes, void *stream) {
    fge_batch *b = nullptr;
    fge_status st = fge_batch_create(n, H, W, p, &b);
    if (st != FGE_OK) return st;
    st = fge_batch_run(b, I, alpha, F, B, workspace, workspace_bytes, stream);
    fge_batch_destroy(b);   // waits for the descriptor upload, not for the kernels
    return st;
}

}  // extern "C"
