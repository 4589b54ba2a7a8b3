// Serving loop (C ABI in include/fge.h): continuous batching of foreground-estimation requests at
// level granularity, with admission by an HBM budget.
//
// A request is one image run through Algorithm 1 with its own level plan, so its F and B are
// bit-identical to fge_estimate_foreground's.  The scheduler thread repeats a tick:
//   1. take newly submitted requests into the FIFO queue,
//   2. retire ticks the device has finished (their last-level requests complete: results are
//      published, workspaces return to the arena, footprints to the budget),
//   3. admit queued requests in arrival order while the budget, the arena and the slot count
//      allow,
//   4. if any request is admitted and a tick slot is free: write the tick's descriptor tables and
//      work lists into the slot's pinned staging buffer, upload them into the slot's arena region
//      (the upload also zeroes the work counters), and enqueue the batched gather and coarse
//      launches for the requests new in this tick, then one persistent tile launch and one
//      persistent streaming launch covering the next fine level of every admitted request, and
//      an event.
// The kernels are the batched kernels of the uneven-batch path; only the schedule differs: there,
// all images' levels are aligned from the finest once; here each request advances one level per
// tick from the tick that admits it, so requests at different levels share launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "fge_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kDefaultMaxActive = 1024;
constexpr int kDefaultDepth = 2;
constexpr int kMaxDepth = 8;
constexpr uint64_t kDefaultTableBytes = 16ull << 20;
constexpr uint64_t kMinTableBytes = 64ull << 10;

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// First-fit allocator over byte offsets of the arena, blocks 256-byte aligned, free neighbours
// merged on release.
class ArenaAlloc {
  public:
    void init(size_t off, size_t bytes) {
        free_.clear();
        if (bytes) free_[off] = bytes;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    const void *I = nullptr, *A = nullptr;
    void *F = nullptr, *B = nullptr;
    fge::Plan plan;
    size_t charge = 0;      // footprint against the budget
    size_t ws_off = 0;      // workspace block in the arena
    int next = -1;          // -1: coarse block not run yet; else the next fine level
    int ticks = 0;
    double submit_ms = 0, admit_ms = 0;
};

struct Slot {
    char *staging = nullptr;   // pinned host image of the tick tables
    size_t dev_off = 0;        // their device copy in the arena
    hipEvent_t done = nullptr;
    std::vector<Request *> finishing;
};

// One fine-level entry of a tick: request, level, work units.
struct Entry {
    Request *r;
    int j;
    int units;
    long px;
};

int tile_units_of(const fge::Level &lv) {
    fge::LevelIO io{};
    io.w = lv.w;
    io.h = lv.h;
    fge::TileArgs a;
    fge::make_tile_args(io, &a);
    return fge::tile_units(a);
}

int fine_units_of(const fge::Level &lv, int strip_rows) {
    fge::LevelIO io{};
    io.w = lv.w;
    io.h = lv.h;
    fge::FineArgs a;
    fge::make_fine_args(io, strip_rows, &a);
    return fge::fine_units(a);
}

// Checks a plan can run on the batched kernels: coarse block first, fused fine levels after.
fge_status batchable(const fge::Plan &pl) {
    if (pl.nc < 1) return FGE_EUNSUPPORTED;
    for (int j = pl.nc; j < pl.n; ++j)
        if (pl.kind[j] != fge::kKindTile && pl.kind[j] != fge::kKindStream) return FGE_EUNSUPPORTED;
    return FGE_OK;
}

size_t footprint(const fge::Plan &pl) {
    return 10 * static_cast<size_t>(pl.W) * pl.H * pl.elem + align256(pl.ws_bytes);
}

// Table bytes one tick needs for this request at its largest step (its first tick, coarse block
// plus first fine level, or a later fine level), alignment included.  Strip counts are taken at
// the lowest strip height a tick can use (8 rows), an upper bound for every height.
size_t max_tick_bytes(const fge::Plan &pl, int strip_rows) {
    if (strip_rows <= 0) strip_rows = 8;
    size_t worst = 0;
    for (int j = pl.nc; j < pl.n; ++j) {
        size_t b = pl.kind[j] == fge::kKindTile
                       ? sizeof(fge::TileArgs) + static_cast<size_t>(tile_units_of(pl.lv[j])) * sizeof(fge::WorkItem)
                       : sizeof(fge::FineArgs) + static_cast<size_t>(fine_units_of(pl.lv[j], strip_rows)) * sizeof(fge::WorkItem);
        if (j == pl.nc) b += sizeof(fge::CoarseArgs) + sizeof(fge::GatherArgs) + sizeof(long long);
        worst = std::max(worst, b);
    }
    return 256 + 8 * 256 + std::max(worst, sizeof(fge::CoarseArgs) + sizeof(fge::GatherArgs) + sizeof(long long));
}

}  // namespace

struct fge_server {
    fge_params prm{};
    fge_server_config cfg{};
    char *arena = nullptr;
    size_t arena_bytes = 0, reserved = 0, budget = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    hipEvent_t start_ev = nullptr;
    Clock::time_point t0;

    // shared with the API threads, guarded by mu
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::deque<Request *> incoming;
    std::deque<fge_server_result> results;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    int error = FGE_OK;
    fge_server_stats stats{};

    // owned by the scheduler thread
    std::thread worker;
    ArenaAlloc alloc;
    size_t charged = 0, arena_used = 0;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::vector<Slot> slots;
    std::deque<int> inflight;       // slot indices, oldest first
    std::vector<int> free_slots;
    double active_sum = 0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    }
};

namespace {

void publish(fge_server *s, std::vector<fge_server_result> &out) {
    if (out.empty()) return;
    std::lock_guard<std::mutex> g(s->mu);
    for (auto &r : out) s->results.push_back(r);
    s->completed += static_cast<int64_t>(out.size());
    s->stats.completed = s->completed;
    out.clear();
    s->cv_idle.notify_all();
}

// The device has finished slot si: complete its requests and free the slot.
fge_status retire(fge_server *s, int si) {
    Slot &sl = s->slots[si];
    float ms = 0.0f;
    const bool ok = hipEventElapsedTime(&ms, s->start_ev, sl.done) == hipSuccess;
    std::vector<fge_server_result> out;
    for (Request *r : sl.finishing) {
        fge_server_result res{};
        res.id = r->id;
        res.status = ok ? FGE_OK : FGE_EHIP;
        res.ticks = r->ticks;
        res.submit_ms = r->submit_ms;
        res.admit_ms = r->admit_ms;
        res.ready_ms = ms;
        res.latency_ms = ms - r->submit_ms;
        out.push_back(res);
        if (r->plan.ws_bytes) s->alloc.release(r->ws_off, r->plan.ws_bytes);
        s->arena_used -= align256(r->plan.ws_bytes);
        s->charged -= r->charge;
        delete r;
    }
    sl.finishing.clear();
    s->free_slots.push_back(si);
    publish(s, out);
    return ok ? FGE_OK : FGE_EHIP;
}

// Retire every finished tick in order; with `block`, wait for the oldest one first.
fge_status retire_done(fge_server *s, bool block) {
    while (!s->inflight.empty()) {
        const int si = s->inflight.front();
        hipError_t e = block ? hipEventSynchronize(s->slots[si].done) : hipEventQuery(s->slots[si].done);
        if (e == hipErrorNotReady) return FGE_OK;
        if (e != hipSuccess) return FGE_EHIP;
        s->inflight.pop_front();
        block = false;
        const fge_status st = retire(s, si);
        if (st != FGE_OK) return st;
    }
    return FGE_OK;
}

void admit(fge_server *s) {
    const size_t max_active = static_cast<size_t>(s->cfg.max_active);
    while (!s->pending.empty() && s->active.size() < max_active) {
        Request *r = s->pending.front();
        if (s->charged + r->charge > s->budget) break;
        size_t off = 0;
        if (r->plan.ws_bytes && !s->alloc.alloc(r->plan.ws_bytes, &off)) break;
        r->ws_off = off;
        r->admit_ms = s->now_ms();
        const bool busy = !s->active.empty() || !s->inflight.empty();
        s->charged += r->charge;
        s->arena_used += align256(r->plan.ws_bytes);
        s->pending.pop_front();
        s->active.push_back(r);
        std::lock_guard<std::mutex> g(s->mu);
        if (busy) ++s->stats.admitted_while_busy;
        s->stats.peak_active = std::max<int32_t>(s->stats.peak_active, static_cast<int32_t>(s->active.size()));
        s->stats.peak_charged_bytes = std::max<uint64_t>(s->stats.peak_charged_bytes, s->charged);
        s->stats.peak_arena_bytes = std::max<uint64_t>(s->stats.peak_arena_bytes, s->reserved + s->arena_used);
    }
}

// Build and enqueue one tick in a free slot.
fge_status enqueue_tick(fge_server *s) {
    const int si = s->free_slots.back();
    Slot &sl = s->slots[si];
    const size_t cap = s->cfg.tick_table_bytes;
    // Strip height of this tick's streaming launch: the caller's, else one for all the streaming
    // levels the admitted requests run next.
    int strip_rows = s->prm.strip_rows;
    if (strip_rows <= 0) {
        std::vector<int> ws, hs;
        for (Request *r : s->active) {
            const int j = r->next < 0 ? r->plan.nc : r->next;
            if (j < r->plan.n && r->plan.kind[j] == fge::kKindStream) {
                ws.push_back(r->plan.lv[j].w);
                hs.push_back(r->plan.lv[j].h);
            }
        }
        strip_rows = fge::launch_strip_rows(ws.data(), hs.data(), static_cast<int>(ws.size()));
    }

    // Select the requests that fit the slot's tables, in admission order.
    std::vector<Request *> fresh;      // run the gather pre-pass and the coarse block
    std::vector<Request *> gathered;   // the subset of fresh with a gather pre-pass
    std::vector<Entry> tile, stream;
    std::vector<Request *> ran;
    size_t need = 256 + 8 * 256;       // counters, alignment of 7 regions
    for (Request *r : s->active) {
        const fge::Plan &pl = r->plan;
        const bool is_new = r->next < 0;
        const int j = is_new ? pl.nc : r->next;
        size_t add = 0;
        if (is_new) {
            add += sizeof(fge::CoarseArgs);
            if (pl.ng > 0) add += sizeof(fge::GatherArgs) + sizeof(long long);
        }
        Entry e{r, j, 0, 0};
        if (j < pl.n) {
            e.px = static_cast<long>(pl.lv[j].w) * pl.lv[j].h;
            if (pl.kind[j] == fge::kKindTile) {
                e.units = tile_units_of(pl.lv[j]);
                add += sizeof(fge::TileArgs);
            } else {
                e.units = fine_units_of(pl.lv[j], strip_rows);
                add += sizeof(fge::FineArgs);
            }
            add += static_cast<size_t>(e.units) * sizeof(fge::WorkItem);
        }
        if (need + add > cap) continue;   // stays for a later tick
        need += add;
        ran.push_back(r);
        if (is_new) {
            fresh.push_back(r);
            if (pl.ng > 0) gathered.push_back(r);
        }
        if (j < pl.n) (pl.kind[j] == fge::kKindTile ? tile : stream).push_back(e);
    }
    if (ran.empty()) return FGE_EINVAL;   // cannot happen: one request's tables fit any capacity
    auto larger = [](const Entry &a, const Entry &b) { return a.px > b.px; };
    std::stable_sort(tile.begin(), tile.end(), larger);
    std::stable_sort(stream.begin(), stream.end(), larger);

    // Lay out and fill the tables (staging image; counters at offset 0 stay zero).
    char *tab = sl.staging;
    std::memset(tab, 0, 256);
    size_t off = 256;
    auto region = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const float om = s->prm.omega, ep = s->prm.eps_r;
    const size_t g_desc = region(gathered.size() * sizeof(fge::GatherArgs));
    const size_t g_first = region(gathered.size() * sizeof(long long));
    long long g_total = 0;
    for (size_t k = 0; k < gathered.size(); ++k) {
        Request *r = gathered[k];
        auto *gd = reinterpret_cast<fge::GatherArgs *>(tab + g_desc) + k;
        fge::make_gather_args(r->plan, r->I, r->A, s->arena + r->ws_off + r->plan.pyr_off, gd);
        reinterpret_cast<long long *>(tab + g_first)[k] = g_total;
        g_total += fge::gather_units(*gd);
    }
    const size_t c_desc = region(fresh.size() * sizeof(fge::CoarseArgs));
    for (size_t k = 0; k < fresh.size(); ++k) {
        Request *r = fresh[k];
        char *ws = s->arena + r->ws_off;
        const fge::LevelSrc src = fge::coarse_src(r->plan, ws, r->F, r->I, r->A);
        void *fo, *bo;
        fge::level_state(r->plan, ws, r->plan.nc - 1, r->F, r->B, &fo, &bo);
        fge::make_coarse_args(r->plan, src, fo, bo, om, ep,
                              reinterpret_cast<fge::CoarseArgs *>(tab + c_desc) + k);
    }
    struct Lay {
        size_t desc, items;
        int nitems;
    };
    auto lay_out = [&](const std::vector<Entry> &es, bool is_tile) {
        Lay L{};
        L.desc = region(es.size() * (is_tile ? sizeof(fge::TileArgs) : sizeof(fge::FineArgs)));
        size_t nit = 0;
        for (const Entry &e : es) nit += static_cast<size_t>(e.units);
        L.items = region(nit * sizeof(fge::WorkItem));
        auto *items = reinterpret_cast<fge::WorkItem *>(tab + L.items);
        int m = 0;
        for (size_t d = 0; d < es.size(); ++d) {
            Request *r = es[d].r;
            const fge::LevelIO io = fge::level_io(r->plan, s->arena + r->ws_off, es[d].j, r->I, r->A,
                                                  r->F, r->B, om, ep);
            if (is_tile)
                fge::make_tile_args(io, reinterpret_cast<fge::TileArgs *>(tab + L.desc) + d);
            else
                fge::make_fine_args(io, strip_rows, reinterpret_cast<fge::FineArgs *>(tab + L.desc) + d);
            for (int u = 0; u < es[d].units; ++u) items[m++] = fge::WorkItem{static_cast<int>(d), u};
        }
        L.nitems = m;
        return L;
    };
    const Lay lt = lay_out(tile, true);
    const Lay ls = lay_out(stream, false);
    const size_t used = off;

    // Enqueue: upload, gather, coarse, tile, streaming, event.
    hipStream_t st = s->stream;
    char *dev = s->arena + sl.dev_off;
    const int storage = s->prm.storage;
    if (hipMemcpyAsync(dev, tab, used, hipMemcpyHostToDevice, st) != hipSuccess) return FGE_EHIP;
    int *cnt = reinterpret_cast<int *>(dev);
    int launches = 0;
    if (!gathered.empty()) {
        if (fge::launch_gather_batch(reinterpret_cast<const fge::GatherArgs *>(dev + g_desc),
                                     reinterpret_cast<const long long *>(dev + g_first),
                                     static_cast<int>(gathered.size()), g_total, storage, st))
            return FGE_EHIP;
        ++launches;
    }
    if (!fresh.empty()) {
        if (fge::launch_coarse_batch(reinterpret_cast<const fge::CoarseArgs *>(dev + c_desc),
                                     static_cast<int>(fresh.size()), storage, st))
            return FGE_EHIP;
        ++launches;
    }
    if (lt.nitems > 0) {
        if (fge::launch_tile_batch(reinterpret_cast<const fge::TileArgs *>(dev + lt.desc),
                                   reinterpret_cast<const fge::WorkItem *>(dev + lt.items),
                                   lt.nitems, cnt, storage, st))
            return FGE_EHIP;
        ++launches;
    }
    if (ls.nitems > 0) {
        if (fge::launch_fine_batch(reinterpret_cast<const fge::FineArgs *>(dev + ls.desc),
                                   reinterpret_cast<const fge::WorkItem *>(dev + ls.items),
                                   ls.nitems, cnt + 1, storage, st))
            return FGE_EHIP;
        ++launches;
    }
    if (hipEventRecord(sl.done, st) != hipSuccess) return FGE_EHIP;
    s->free_slots.pop_back();
    s->inflight.push_back(si);

    // Advance the requests that ran; the ones past their last level finish with this tick.
    std::vector<int> levels;
    for (Request *r : ran) {
        levels.push_back(r->next < 0 ? -1 : r->next);
        if (r->next < 0) {
            r->next = r->plan.nc;
            if (r->next < r->plan.n) levels.push_back(r->next);
        }
        if (r->next < r->plan.n) ++r->next;
        ++r->ticks;
    }
    std::sort(levels.begin(), levels.end());
    const bool mixed = std::unique(levels.begin(), levels.end()) - levels.begin() > 1;
    for (Request *r : ran)
        if (r->next >= r->plan.n) sl.finishing.push_back(r);
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                   [](Request *r) { return r->next >= r->plan.n; }),
                    s->active.end());
    s->active_sum += static_cast<double>(ran.size());
    std::lock_guard<std::mutex> g(s->mu);
    ++s->stats.ticks;
    s->stats.launches += launches + 1;   // the upload counts as one
    if (mixed) ++s->stats.mixed_ticks;
    s->stats.mean_active = s->active_sum / static_cast<double>(s->stats.ticks);
    return FGE_OK;
}

// After a failure: every request not yet completed completes with the error.
void fail_all(fge_server *s, int err) {
    std::vector<fge_server_result> out;
    auto fail = [&](Request *r) {
        fge_server_result res{};
        res.id = r->id;
        res.status = err;
        res.ticks = r->ticks;
        res.submit_ms = r->submit_ms;
        res.admit_ms = r->admit_ms;
        out.push_back(res);
        delete r;
    };
    (void)hipStreamSynchronize(s->stream);
    for (int si : s->inflight) {
        for (Request *r : s->slots[si].finishing) fail(r);
        s->slots[si].finishing.clear();
        s->free_slots.push_back(si);
    }
    s->inflight.clear();
    for (Request *r : s->active) fail(r);
    s->active.clear();
    for (Request *r : s->pending) fail(r);
    s->pending.clear();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->error = err;
        for (Request *r : s->incoming) fail(r);
        s->incoming.clear();
    }
    publish(s, out);
}

void worker_main(fge_server *s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        fail_all(s, FGE_EHIP);
        std::unique_lock<std::mutex> g(s->mu);
        s->cv_work.wait(g, [&] { return s->stop; });
        return;
    }
    for (;;) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            while (!s->incoming.empty()) {
                s->pending.push_back(s->incoming.front());
                s->incoming.pop_front();
            }
        }
        fge_status st = retire_done(s, false);
        if (st == FGE_OK) {
            admit(s);
            if (!s->active.empty()) {
                st = s->free_slots.empty() ? retire_done(s, true) : enqueue_tick(s);
                if (st == FGE_OK) continue;
            }
        }
        if (st != FGE_OK) {
            fail_all(s, st);
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return s->stop; });
            return;
        }
        if (!s->inflight.empty()) {   // the device is busy and nothing can be enqueued: poll
            std::this_thread::yield();
            continue;
        }
        if (!s->pending.empty()) {    // idle device, empty arena, and the head does not fit:
            fail_all(s, FGE_EBUDGET); // excluded by the checks in fge_server_submit
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return s->stop; });
            return;
        }
        std::unique_lock<std::mutex> g(s->mu);
        if (s->stop && s->incoming.empty() && s->pending.empty()) return;
        s->cv_work.wait(g, [&] { return s->stop || !s->incoming.empty(); });
    }
}

fge_status request_plan(const fge_params &p, int W, int H, fge::Plan *pl) {
    const fge_status st = fge::make_plan(W, H, p, pl);
    if (st != FGE_OK) return st;
    return batchable(*pl);
}

}  // namespace

extern "C" {

void fge_server_default_config(fge_server_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->size = sizeof(fge_server_config);
    c->max_active = kDefaultMaxActive;
    c->pipeline_depth = kDefaultDepth;
    c->budget_bytes = 0;
    c->tick_table_bytes = kDefaultTableBytes;
}

size_t fge_server_request_bytes(int32_t H, int32_t W, const fge_params *p) {
    fge_params prm;
    if (p) prm = *p; else fge_default_params(&prm);
    fge::Plan pl;
    if (fge::make_plan(W, H, prm, &pl) != FGE_OK) return 0;
    return footprint(pl);
}

size_t fge_server_reserved_bytes(const fge_server_config *c) {
    fge_server_config cfg;
    if (c) cfg = *c; else fge_server_default_config(&cfg);
    const int depth = cfg.pipeline_depth ? cfg.pipeline_depth : kDefaultDepth;
    const uint64_t tab = cfg.tick_table_bytes ? cfg.tick_table_bytes : kDefaultTableBytes;
    return static_cast<size_t>(depth) * align256(tab);
}

fge_status fge_server_create(const fge_params *p, const fge_server_config *c, void *arena,
                             size_t arena_bytes, void *stream, fge_server **out) {
    if (!out) return FGE_EINVAL;
    *out = nullptr;
    fge_params prm;
    if (p) prm = *p; else fge_default_params(&prm);
    if (!fge::params_valid(prm)) return FGE_EINVAL;
    if (prm.kernel == FGE_KERNEL_NAIVE || prm.coarse_max_px < 0 || prm.iters_big != 2 ||
        prm.order != FGE_REDBLACK)
        return FGE_EUNSUPPORTED;
    fge_server_config cfg;
    if (c) cfg = *c; else fge_server_default_config(&cfg);
    if (cfg.size != sizeof(fge_server_config)) return FGE_EINVAL;
    if (cfg.max_active == 0) cfg.max_active = kDefaultMaxActive;
    if (cfg.pipeline_depth == 0) cfg.pipeline_depth = kDefaultDepth;
    if (cfg.tick_table_bytes == 0) cfg.tick_table_bytes = kDefaultTableBytes;
    if (cfg.max_active < 1 || cfg.max_active > (1 << 16) || cfg.pipeline_depth < 1 ||
        cfg.pipeline_depth > kMaxDepth || cfg.tick_table_bytes < kMinTableBytes ||
        cfg.tick_table_bytes > (1ull << 32))
        return FGE_EINVAL;
    cfg.tick_table_bytes = align256(cfg.tick_table_bytes);
    if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) || !stream) return FGE_EINVAL;
    const size_t reserved = fge_server_reserved_bytes(&cfg);
    if (arena_bytes <= reserved) return FGE_EWORKSPACE;
    if (cfg.budget_bytes == 0) cfg.budget_bytes = arena_bytes;

    fge_server *s = new (std::nothrow) fge_server();
    if (!s) return FGE_ENOMEM;
    s->prm = prm;
    s->cfg = cfg;
    s->arena = static_cast<char *>(arena);
    s->arena_bytes = arena_bytes;
    s->reserved = reserved;
    s->budget = cfg.budget_bytes;
    s->stream = static_cast<hipStream_t>(stream);
    s->alloc.init(reserved, (arena_bytes - reserved) & ~static_cast<size_t>(255));
    bool ok = hipGetDevice(&s->device) == hipSuccess && hipEventCreate(&s->start_ev) == hipSuccess;
    s->slots.resize(cfg.pipeline_depth);
    for (int k = 0; ok && k < cfg.pipeline_depth; ++k) {
        Slot &sl = s->slots[k];
        sl.dev_off = static_cast<size_t>(k) * cfg.tick_table_bytes;
        ok = hipHostMalloc(reinterpret_cast<void **>(&sl.staging), cfg.tick_table_bytes,
                           hipHostMallocDefault) == hipSuccess &&
             hipEventCreate(&sl.done) == hipSuccess;
        s->free_slots.push_back(cfg.pipeline_depth - 1 - k);
    }
    // Time origin: the start event on the idle stream, and the host clock right after it.
    ok = ok && hipStreamSynchronize(s->stream) == hipSuccess &&
         hipEventRecord(s->start_ev, s->stream) == hipSuccess &&
         hipEventSynchronize(s->start_ev) == hipSuccess;
    if (!ok) {
        fge_server_destroy(s);
        return FGE_EHIP;
    }
    s->t0 = Clock::now();
    s->worker = std::thread(worker_main, s);
    *out = s;
    return FGE_OK;
}

fge_status fge_server_submit(fge_server *s, int64_t id, const void *I, const void *alpha,
                             int32_t H, int32_t W, void *F, void *B) {
    if (!s || !I || !alpha || !F || !B) return FGE_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return FGE_ENOMEM;
    const fge_status st = request_plan(s->prm, W, H, &r->plan);
    if (st != FGE_OK) {
        delete r;
        return st;
    }
    if (fge::outputs_alias(I, alpha, F, B, W, H, r->plan.elem, s->arena, s->arena_bytes)) {
        delete r;
        return FGE_EINVAL;
    }
    r->charge = footprint(r->plan);
    if (r->charge > s->budget || max_tick_bytes(r->plan, s->prm.strip_rows) > s->cfg.tick_table_bytes ||
        align256(r->plan.ws_bytes) > ((s->arena_bytes - s->reserved) & ~static_cast<size_t>(255))) {
        delete r;
        return FGE_EBUDGET;
    }
    r->id = id;
    r->I = I;
    r->A = alpha;
    r->F = F;
    r->B = B;
    r->submit_ms = s->now_ms();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error != FGE_OK) {
        delete r;
        return static_cast<fge_status>(s->error);
    }
    if (s->stop) {
        delete r;
        return FGE_EINVAL;
    }
    s->incoming.push_back(r);
    ++s->submitted;
    s->stats.submitted = s->submitted;
    s->cv_work.notify_one();
    return FGE_OK;
}

int32_t fge_server_poll(fge_server *s, fge_server_result *out, int32_t cap) {
    if (!s || (cap > 0 && !out) || cap < 0) return FGE_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    int32_t k = 0;
    while (k < cap && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    if (k == 0 && s->error != FGE_OK) return s->error;
    return k;
}

fge_status fge_server_drain(fge_server *s) {
    if (!s) return FGE_EINVAL;
    std::unique_lock<std::mutex> g(s->mu);
    s->cv_idle.wait(g, [&] { return s->completed >= s->submitted; });
    return static_cast<fge_status>(s->error);
}

fge_status fge_server_get_stats(fge_server *s, fge_server_stats *out) {
    if (!s || !out) return FGE_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return FGE_OK;
}

void fge_server_destroy(fge_server *s) {
    if (!s) return;
    if (s->worker.joinable()) {
        fge_server_drain(s);
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
            s->cv_work.notify_all();
        }
        s->worker.join();
    }
    for (Slot &sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.staging) (void)hipHostFree(sl.staging);
    }
    if (s->start_ev) (void)hipEventDestroy(s->start_ev);
    delete s;
}

}  // extern "C"
