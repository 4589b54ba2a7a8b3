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
//
// The scheduler talks to the device through an executor: the HIP one (pinned staging, the
// server's stream, an event per tick slot) or a host model of it (fge_server_create_simulated:
// modelled tick durations, injectable launch and device failures, and a manual mode in which the
// caller's thread runs the scheduler step by step), which the CPU tests and sanitizer builds drive.
// Failures: a tick whose launch fails fails only the requests in that tick (after everything
// already enqueued has finished) and the server goes on; an error reported by the device itself
// fails every request not yet completed and ends the server.  Queued requests (not yet admitted)
// can be cancelled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
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

namespace fge {
namespace serve {

// What one tick asks of the device: the size of its tables and where each launch's descriptors
// and work items sit, as byte offsets from the slot's table base.
struct TickWork {
    size_t bytes = 0;
    size_t g_desc = 0, g_first = 0;
    int n_gather = 0;
    long long g_total = 0;
    size_t c_desc = 0;
    int n_coarse = 0;
    size_t t_desc = 0, t_items = 0;
    int t_n = 0;
    size_t s_desc = 0, s_items = 0;
    int s_n = 0;
    long long px = 0;   // fine-level pixels the tick advances (the simulated executor's cost)
};

// The device side of a server.  The scheduler owns the schedule (admission, the tick tables, the
// arena); an executor uploads a tick's tables, runs its launches and reports completion.  Slots
// 0 .. depth-1 each hold one tick at a time; ticks complete in the order they were launched.
class Executor {
  public:
    virtual ~Executor() = default;
    virtual fge_status init(int depth, size_t table_bytes) = 0;
    virtual char *staging(int slot) = 0;             // host image of the slot's tables
    virtual fge_status start_clock() = 0;            // time origin of now_ms and ready times
    virtual double now_ms() = 0;                     // host clock, ms after the origin
    virtual fge_status bind_thread() = 0;            // on the scheduler thread, before any launch
    // Upload the slot's tables to `dev` and enqueue the tick's launches and completion marker.
    // After a failure, an unknown part of the tick may have been enqueued.
    virtual fge_status launch(int slot, char *dev, const TickWork &w, int *launches) = 0;
    // 1: the slot's tick is done (*ready_ms: device completion time); 0: not yet; < 0: an error of
    // the device itself (the server cannot go on).
    virtual int poll(int slot, bool block, double *ready_ms) = 0;
    virtual void quiesce() = 0;                      // wait for everything enqueued so far
};

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// The MI355X: pinned staging and an event per slot, every launch on the server's stream.
class HipExecutor final : public Executor {
  public:
    HipExecutor(hipStream_t stream, int storage) : stream_(stream), storage_(storage) {}
    ~HipExecutor() override {
        for (Slot &sl : slots_) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.staging) (void)hipHostFree(sl.staging);
        }
        if (start_) (void)hipEventDestroy(start_);
    }
    fge_status init(int depth, size_t table_bytes) override {
        if (hipGetDevice(&device_) != hipSuccess || hipEventCreate(&start_) != hipSuccess)
            return FGE_EHIP;
        slots_.resize(depth);
        for (Slot &sl : slots_)
            if (hipHostMalloc(reinterpret_cast<void **>(&sl.staging), table_bytes,
                              hipHostMallocDefault) != hipSuccess ||
                hipEventCreate(&sl.done) != hipSuccess)
                return FGE_EHIP;
        return FGE_OK;
    }
    char *staging(int slot) override { return slots_[slot].staging; }
    fge_status start_clock() override {
        // the start event on the idle stream, and the host clock right after it
        if (hipStreamSynchronize(stream_) != hipSuccess || hipEventRecord(start_, stream_) != hipSuccess ||
            hipEventSynchronize(start_) != hipSuccess)
            return FGE_EHIP;
        t0_ = Clock::now();
        return FGE_OK;
    }
    double now_ms() override { return ms_since(t0_); }
    fge_status bind_thread() override {
        return hipSetDevice(device_) == hipSuccess ? FGE_OK : FGE_EHIP;
    }
    fge_status launch(int slot, char *dev, const TickWork &w, int *launches) override {
        *launches = 0;
        hipStream_t st = stream_;
        if (hipMemcpyAsync(dev, slots_[slot].staging, w.bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return FGE_EHIP;
        int *cnt = reinterpret_cast<int *>(dev);   // the tile and the streaming launch's queues
        if (w.n_gather > 0) {
            if (launch_gather_batch(reinterpret_cast<const GatherArgs *>(dev + w.g_desc),
                                    reinterpret_cast<const long long *>(dev + w.g_first), w.n_gather,
                                    w.g_total, storage_, st))
                return FGE_EHIP;
            ++*launches;
        }
        if (w.n_coarse > 0) {
            if (launch_coarse_batch(reinterpret_cast<const CoarseArgs *>(dev + w.c_desc), w.n_coarse,
                                    storage_, st))
                return FGE_EHIP;
            ++*launches;
        }
        if (w.t_n > 0) {
            if (launch_tile_batch(reinterpret_cast<const TileArgs *>(dev + w.t_desc),
                                  reinterpret_cast<const WorkItem *>(dev + w.t_items), w.t_n, cnt,
                                  storage_, st))
                return FGE_EHIP;
            ++*launches;
        }
        if (w.s_n > 0) {
            if (launch_fine_batch(reinterpret_cast<const FineArgs *>(dev + w.s_desc),
                                  reinterpret_cast<const WorkItem *>(dev + w.s_items), w.s_n,
                                  cnt + kQueueCounters,
                                  storage_, st))
                return FGE_EHIP;
            ++*launches;
        }
        return hipEventRecord(slots_[slot].done, st) == hipSuccess ? FGE_OK : FGE_EHIP;
    }
    int poll(int slot, bool block, double *ready_ms) override {
        hipEvent_t e = slots_[slot].done;
        const hipError_t r = block ? hipEventSynchronize(e) : hipEventQuery(e);
        if (r == hipErrorNotReady) return 0;
        float ms = 0.0f;
        if (r != hipSuccess || hipEventElapsedTime(&ms, start_, e) != hipSuccess) return FGE_EHIP;
        *ready_ms = ms;
        return 1;
    }
    void quiesce() override { (void)hipStreamSynchronize(stream_); }

  private:
    struct Slot {
        char *staging = nullptr;
        hipEvent_t done = nullptr;
    };
    hipStream_t stream_;
    int storage_;
    int device_ = 0;
    hipEvent_t start_ = nullptr;
    Clock::time_point t0_;
    std::vector<Slot> slots_;
};

// A host model of the device for the scheduler's tests: nothing is uploaded or launched and no
// buffer is touched; a tick takes us_per_launch per launch plus us_per_mpx per megapixel of its
// fine levels, ticks run one after another.  Manual mode: the clock and the completions move only
// when the caller says so (fge_server_sim_step), so every schedule is reproducible.
class SimExecutor final : public Executor {
  public:
    explicit SimExecutor(const fge_server_sim &c) : cfg_(c) {}
    fge_status init(int depth, size_t table_bytes) override {
        slots_.resize(depth);
        for (Slot &sl : slots_) sl.staging.assign(table_bytes, 0);
        return FGE_OK;
    }
    char *staging(int slot) override { return slots_[slot].staging.data(); }
    fge_status start_clock() override {
        std::lock_guard<std::mutex> g(mu_);
        t0_ = Clock::now();
        clock_ = 0.0;
        return FGE_OK;
    }
    double now_ms() override {
        std::lock_guard<std::mutex> g(mu_);
        return cfg_.manual ? clock_ : ms_since(t0_);
    }
    fge_status bind_thread() override { return FGE_OK; }
    fge_status launch(int slot, char *, const TickWork &w, int *launches) override {
        std::lock_guard<std::mutex> g(mu_);
        const int k = ++ticks_;
        *launches = 0;
        if (k == cfg_.fail_launch_tick) return FGE_EHIP;
        *launches = (w.n_gather > 0) + (w.n_coarse > 0) + (w.t_n > 0) + (w.s_n > 0);
        Slot &sl = slots_[slot];
        sl.busy = true;
        sl.done = false;
        sl.fail = k == cfg_.fail_device_tick;
        const double cost_ms = (cfg_.us_per_launch * (*launches + 1) +
                                cfg_.us_per_mpx * static_cast<double>(w.px) * 1e-6) * 1e-3;
        const double begin = std::max(cfg_.manual ? clock_ : ms_since(t0_), last_end_);
        sl.end = begin + cost_ms;
        last_end_ = sl.end;
        order_.push_back(slot);
        return FGE_OK;
    }
    int poll(int slot, bool block, double *ready_ms) override {
        std::unique_lock<std::mutex> g(mu_);
        Slot &sl = slots_[slot];
        if (!sl.busy) return 0;
        if (cfg_.manual) {
            if (!sl.done) return 0;
        } else {
            const double wait = sl.end - ms_since(t0_);
            if (wait > 0.0) {
                if (!block) return 0;
                g.unlock();
                std::this_thread::sleep_for(std::chrono::duration<double, std::milli>(wait));
                g.lock();
            }
            if (!order_.empty() && order_.front() == slot) order_.pop_front();
        }
        if (sl.fail) return FGE_EHIP;
        *ready_ms = sl.end;
        sl.busy = false;
        return 1;
    }
    void quiesce() override {}
    // Manual mode: move the clock, then complete the oldest `n` ticks at their modelled end or
    // the clock, whichever is later.
    void step(int n, double advance_ms) {
        std::lock_guard<std::mutex> g(mu_);
        clock_ += advance_ms;
        for (; n > 0 && !order_.empty(); --n) {
            Slot &sl = slots_[order_.front()];
            order_.pop_front();
            sl.end = std::max(sl.end, clock_);
            clock_ = sl.end;
            sl.done = true;
        }
    }
    int outstanding() {
        std::lock_guard<std::mutex> g(mu_);
        return static_cast<int>(order_.size());
    }

  private:
    struct Slot {
        std::vector<char> staging;
        bool busy = false, done = false, fail = false;
        double end = 0.0;
    };
    fge_server_sim cfg_;
    std::mutex mu_;
    Clock::time_point t0_ = Clock::now();
    double clock_ = 0.0, last_end_ = 0.0;
    int ticks_ = 0;
    std::deque<int> order_;   // launched, not yet completed (manual) / not yet polled (auto)
    std::vector<Slot> slots_;
};

struct Slot {
    size_t dev_off = 0;                 // the slot's tick tables in the arena
    std::vector<Request *> finishing;   // requests whose last level is in this tick
};

}  // namespace serve
}  // namespace fge

struct fge_server {
    fge_params prm{};
    fge_server_config cfg{};
    char *arena = nullptr;
    size_t arena_bytes = 0, reserved = 0, budget = 0;
    std::unique_ptr<fge::serve::Executor> exec;
    fge::serve::SimExecutor *sim = nullptr;   // exec, when simulated
    bool manual = false;                      // simulated, driven by fge_server_sim_step
    std::mutex step_mu;                       // one manual driver at a time

    // shared with the API threads, guarded by mu
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::deque<Request *> incoming;
    std::deque<Request *> pending;   // taken in by the scheduler, not admitted yet (cancellable)
    std::deque<fge_server_result> results;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    int error = FGE_OK;
    fge_server_stats stats{};

    // owned by the scheduler
    std::thread worker;
    ArenaAlloc alloc;
    size_t charged = 0, arena_used = 0;
    std::vector<Request *> active;
    std::vector<fge::serve::Slot> slots;
    std::deque<int> inflight;       // slot indices, oldest first
    std::vector<int> free_slots;
    double active_sum = 0;
};

namespace {

using fge::serve::TickWork;

fge_server_result make_result(const Request *r, int status, double ready_ms) {
    fge_server_result res{};
    res.id = r->id;
    res.status = status;
    res.ticks = r->ticks;
    res.submit_ms = r->submit_ms;
    res.admit_ms = r->admit_ms;
    res.ready_ms = ready_ms;
    res.latency_ms = ready_ms - r->submit_ms;
    return res;
}

void publish(fge_server *s, std::vector<fge_server_result> &out, int64_t failed = 0) {
    if (out.empty()) return;
    std::lock_guard<std::mutex> g(s->mu);
    for (auto &r : out) s->results.push_back(r);
    s->completed += static_cast<int64_t>(out.size());
    s->stats.completed = s->completed;
    s->stats.failed += failed;
    out.clear();
    s->cv_idle.notify_all();
}

// A request leaves the device: its workspace returns to the arena, its footprint to the budget.
void release(fge_server *s, Request *r) {
    if (r->plan.ws_bytes) s->alloc.release(r->ws_off, r->plan.ws_bytes);
    s->arena_used -= align256(r->plan.ws_bytes);
    s->charged -= r->charge;
}

// The device has finished slot si at ready_ms: complete its requests and free the slot.
void retire(fge_server *s, int si, double ready_ms) {
    fge::serve::Slot &sl = s->slots[si];
    std::vector<fge_server_result> out;
    for (Request *r : sl.finishing) {
        out.push_back(make_result(r, FGE_OK, ready_ms));
        release(s, r);
        delete r;
    }
    sl.finishing.clear();
    s->free_slots.push_back(si);
    publish(s, out);
}

// Retire every finished tick in order; with `block`, wait for the oldest one first.
fge_status retire_done(fge_server *s, bool block) {
    while (!s->inflight.empty()) {
        const int si = s->inflight.front();
        double ready = 0.0;
        const int r = s->exec->poll(si, block, &ready);
        if (r == 0) return FGE_OK;
        if (r < 0) return static_cast<fge_status>(r);
        s->inflight.pop_front();
        block = false;
        retire(s, si, ready);
    }
    return FGE_OK;
}

void admit(fge_server *s) {
    const size_t max_active = static_cast<size_t>(s->cfg.max_active);
    std::lock_guard<std::mutex> g(s->mu);
    while (!s->pending.empty() && s->active.size() < max_active) {
        Request *r = s->pending.front();
        if (s->charged + r->charge > s->budget) break;
        size_t off = 0;
        if (r->plan.ws_bytes && !s->alloc.alloc(r->plan.ws_bytes, &off)) break;
        r->ws_off = off;
        r->admit_ms = s->exec->now_ms();
        const bool busy = !s->active.empty() || !s->inflight.empty();
        s->charged += r->charge;
        s->arena_used += align256(r->plan.ws_bytes);
        s->pending.pop_front();
        s->active.push_back(r);
        if (busy) ++s->stats.admitted_while_busy;
        s->stats.peak_active = std::max<int32_t>(s->stats.peak_active, static_cast<int32_t>(s->active.size()));
        s->stats.peak_charged_bytes = std::max<uint64_t>(s->stats.peak_charged_bytes, s->charged);
        s->stats.peak_arena_bytes = std::max<uint64_t>(s->stats.peak_arena_bytes, s->reserved + s->arena_used);
    }
}

// A tick whose launch failed: its requests fail with the error and leave the server, the rest go
// on.  Everything already enqueued is waited for first, so no launch still uses their memory.
void fail_tick(fge_server *s, const std::vector<Request *> &ran, int err) {
    s->exec->quiesce();
    const double now = s->exec->now_ms();
    std::vector<fge_server_result> out;
    for (Request *r : ran) {
        out.push_back(make_result(r, err, now));
        release(s, r);
        s->active.erase(std::remove(s->active.begin(), s->active.end(), r), s->active.end());
        delete r;
    }
    publish(s, out, static_cast<int64_t>(ran.size()));
}

// Build one tick in a free slot and hand it to the executor.  A failed launch fails the tick's
// requests only (fail_tick) and returns FGE_OK; other errors are the server's.
fge_status enqueue_tick(fge_server *s) {
    const int si = s->free_slots.back();
    fge::serve::Slot &sl = s->slots[si];
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
    char *tab = s->exec->staging(si);
    std::memset(tab, 0, 256);
    size_t off = 256;
    auto region = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    TickWork w;
    const float om = s->prm.omega, ep = s->prm.eps_r;
    w.g_desc = region(gathered.size() * sizeof(fge::GatherArgs));
    w.g_first = region(gathered.size() * sizeof(long long));
    for (size_t k = 0; k < gathered.size(); ++k) {
        Request *r = gathered[k];
        auto *gd = reinterpret_cast<fge::GatherArgs *>(tab + w.g_desc) + k;
        fge::make_gather_args(r->plan, r->I, r->A, s->arena + r->ws_off + r->plan.pyr_off, gd);
        reinterpret_cast<long long *>(tab + w.g_first)[k] = w.g_total;
        w.g_total += fge::gather_units(*gd);
    }
    w.n_gather = static_cast<int>(gathered.size());
    w.c_desc = region(fresh.size() * sizeof(fge::CoarseArgs));
    for (size_t k = 0; k < fresh.size(); ++k) {
        Request *r = fresh[k];
        char *ws = s->arena + r->ws_off;
        const fge::LevelSrc src = fge::coarse_src(r->plan, ws, r->F, r->I, r->A);
        void *fo, *bo;
        fge::level_state(r->plan, ws, r->plan.nc - 1, r->F, r->B, &fo, &bo);
        fge::make_coarse_args(r->plan, src, fo, bo, om, ep,
                              reinterpret_cast<fge::CoarseArgs *>(tab + w.c_desc) + k);
    }
    w.n_coarse = static_cast<int>(fresh.size());
    auto lay_out = [&](const std::vector<Entry> &es, bool is_tile, size_t *desc, size_t *items_at) {
        *desc = region(es.size() * (is_tile ? sizeof(fge::TileArgs) : sizeof(fge::FineArgs)));
        size_t nit = 0;
        for (const Entry &e : es) nit += static_cast<size_t>(e.units);
        *items_at = region(nit * sizeof(fge::WorkItem));
        auto *items = reinterpret_cast<fge::WorkItem *>(tab + *items_at);
        int m = 0;
        for (size_t d = 0; d < es.size(); ++d) {
            Request *r = es[d].r;
            const fge::LevelIO io = fge::level_io(r->plan, s->arena + r->ws_off, es[d].j, r->I, r->A,
                                                  r->F, r->B, om, ep);
            if (is_tile)
                fge::make_tile_args(io, reinterpret_cast<fge::TileArgs *>(tab + *desc) + d);
            else
                fge::make_fine_args(io, strip_rows, reinterpret_cast<fge::FineArgs *>(tab + *desc) + d);
            for (int u = 0; u < es[d].units; ++u) items[m++] = fge::WorkItem{static_cast<int>(d), u};
            w.px += es[d].px;
        }
        return m;
    };
    w.t_n = lay_out(tile, true, &w.t_desc, &w.t_items);
    w.s_n = lay_out(stream, false, &w.s_desc, &w.s_items);
    w.bytes = off;

    int launches = 0;
    const fge_status st = s->exec->launch(si, s->arena + sl.dev_off, w, &launches);
    if (st != FGE_OK) {
        fail_tick(s, ran, st);
        return FGE_OK;
    }
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

// After an error of the device itself: every request not yet completed completes with the error,
// and the server accepts nothing more.
void fail_all(fge_server *s, int err) {
    std::vector<fge_server_result> out;
    const double now = s->exec->now_ms();
    auto fail = [&](Request *r) {
        fge_server_result res = make_result(r, err, now);
        out.push_back(res);
        delete r;
    };
    s->exec->quiesce();
    for (int si : s->inflight) {
        for (Request *r : s->slots[si].finishing) fail(r);
        s->slots[si].finishing.clear();
        s->free_slots.push_back(si);
    }
    s->inflight.clear();
    for (Request *r : s->active) fail(r);
    s->active.clear();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->error = err;
        for (Request *r : s->pending) fail(r);
        s->pending.clear();
        for (Request *r : s->incoming) fail(r);
        s->incoming.clear();
    }
    publish(s, out, static_cast<int64_t>(out.size()));
}

// One pass of the scheduler: take new submissions, retire finished ticks, admit, enqueue one
// tick.  kBusy: requests wait for the device (no free slot, or ticks in flight).
enum Pass { kIdle, kProgress, kBusy, kFatal };

Pass pass(fge_server *s) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        while (!s->incoming.empty()) {
            s->pending.push_back(s->incoming.front());
            s->incoming.pop_front();
        }
    }
    fge_status st = retire_done(s, false);
    if (st != FGE_OK) {
        fail_all(s, st);
        return kFatal;
    }
    admit(s);
    if (!s->active.empty()) {
        if (s->free_slots.empty()) return kBusy;
        st = enqueue_tick(s);
        if (st != FGE_OK) {
            fail_all(s, st);
            return kFatal;
        }
        return kProgress;
    }
    if (!s->inflight.empty()) return kBusy;
    bool waiting;
    {
        std::lock_guard<std::mutex> g(s->mu);
        waiting = !s->pending.empty();
    }
    if (waiting) {   // idle device, empty arena, and the head does not fit:
        fail_all(s, FGE_EBUDGET);   // excluded by the checks in fge_server_submit
        return kFatal;
    }
    return kIdle;
}

void wait_for_stop(fge_server *s) {
    std::unique_lock<std::mutex> g(s->mu);
    s->cv_work.wait(g, [&] { return s->stop; });
}

void worker_main(fge_server *s) {
    if (s->exec->bind_thread() != FGE_OK) {
        fail_all(s, FGE_EHIP);
        wait_for_stop(s);
        return;
    }
    for (;;) {
        const Pass r = pass(s);
        if (r == kFatal) {
            wait_for_stop(s);
            return;
        }
        if (r == kProgress) continue;
        if (r == kBusy) {
            if (!s->active.empty() && s->free_slots.empty()) {   // wait for the oldest tick
                const fge_status st = retire_done(s, true);
                if (st != FGE_OK) {
                    fail_all(s, st);
                    wait_for_stop(s);
                    return;
                }
            } else {
                std::this_thread::yield();   // ticks in flight, nothing to enqueue: poll
            }
            continue;
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

// Checks shared by both kinds of server; fills *prm and *cfg with the defaults applied.
fge_status check_config(const fge_params *p, const fge_server_config *c, size_t arena_bytes,
                        fge_params *prm, fge_server_config *cfg) {
    if (p) *prm = *p; else fge_default_params(prm);
    if (!fge::params_valid(*prm)) return FGE_EINVAL;
    if (prm->kernel == FGE_KERNEL_NAIVE || prm->coarse_max_px < 0 || prm->iters_big != 2 ||
        prm->order != FGE_REDBLACK)
        return FGE_EUNSUPPORTED;
    if (c) *cfg = *c; else fge_server_default_config(cfg);
    if (cfg->size != sizeof(fge_server_config)) return FGE_EINVAL;
    if (cfg->max_active == 0) cfg->max_active = kDefaultMaxActive;
    if (cfg->pipeline_depth == 0) cfg->pipeline_depth = kDefaultDepth;
    if (cfg->tick_table_bytes == 0) cfg->tick_table_bytes = kDefaultTableBytes;
    if (cfg->max_active < 1 || cfg->max_active > (1 << 16) || cfg->pipeline_depth < 1 ||
        cfg->pipeline_depth > kMaxDepth || cfg->tick_table_bytes < kMinTableBytes ||
        cfg->tick_table_bytes > (1ull << 32))
        return FGE_EINVAL;
    cfg->tick_table_bytes = align256(cfg->tick_table_bytes);
    if (arena_bytes <= fge_server_reserved_bytes(cfg)) return FGE_EWORKSPACE;
    if (cfg->budget_bytes == 0) cfg->budget_bytes = arena_bytes;
    return FGE_OK;
}

fge_status create_with(const fge_params &prm, const fge_server_config &cfg, char *arena,
                       size_t arena_bytes, std::unique_ptr<fge::serve::Executor> exec,
                       fge::serve::SimExecutor *sim, bool manual, fge_server **out) {
    fge_server *s = new (std::nothrow) fge_server();
    if (!s) return FGE_ENOMEM;
    s->prm = prm;
    s->cfg = cfg;
    s->arena = arena;
    s->arena_bytes = arena_bytes;
    s->reserved = fge_server_reserved_bytes(&cfg);
    s->budget = cfg.budget_bytes;
    s->exec = std::move(exec);
    s->sim = sim;
    s->manual = manual;
    s->alloc.init(s->reserved, (arena_bytes - s->reserved) & ~static_cast<size_t>(255));
    s->slots.resize(cfg.pipeline_depth);
    for (int k = 0; k < cfg.pipeline_depth; ++k) {
        s->slots[k].dev_off = static_cast<size_t>(k) * cfg.tick_table_bytes;
        s->free_slots.push_back(cfg.pipeline_depth - 1 - k);
    }
    if (s->exec->init(cfg.pipeline_depth, cfg.tick_table_bytes) != FGE_OK ||
        s->exec->start_clock() != FGE_OK) {
        fge_server_destroy(s);
        return FGE_EHIP;
    }
    if (!manual) s->worker = std::thread(worker_main, s);
    *out = s;
    return FGE_OK;
}

// Base address of a simulated server's arena: a range of the address space no host or device
// allocation uses, never dereferenced (descriptors are built but nothing runs).
char *const kSimArena = reinterpret_cast<char *>(static_cast<uintptr_t>(1) << 46);

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
    fge_server_config cfg;
    const fge_status st = check_config(p, c, arena_bytes, &prm, &cfg);
    if (st != FGE_OK) return st;
    if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) || !stream) return FGE_EINVAL;
    std::unique_ptr<fge::serve::Executor> exec(
        new (std::nothrow) fge::serve::HipExecutor(static_cast<hipStream_t>(stream), prm.storage));
    if (!exec) return FGE_ENOMEM;
    return create_with(prm, cfg, static_cast<char *>(arena), arena_bytes, std::move(exec), nullptr,
                       false, out);
}

void fge_server_sim_default(fge_server_sim *m) {
    if (!m) return;
    std::memset(m, 0, sizeof(*m));
    m->size = sizeof(fge_server_sim);
    m->manual = 1;
    m->us_per_launch = 3.0;
    m->us_per_mpx = 8.0;
}

fge_status fge_server_create_simulated(const fge_params *p, const fge_server_config *c,
                                       size_t arena_bytes, const fge_server_sim *m,
                                       fge_server **out) {
    if (!out) return FGE_EINVAL;
    *out = nullptr;
    fge_server_sim sim;
    if (m) sim = *m; else fge_server_sim_default(&sim);
    if (sim.size != sizeof(fge_server_sim) || (sim.manual != 0 && sim.manual != 1) ||
        !(sim.us_per_launch >= 0.0) || !(sim.us_per_mpx >= 0.0) || sim.fail_launch_tick < 0 ||
        sim.fail_device_tick < 0)
        return FGE_EINVAL;
    if (arena_bytes > (static_cast<size_t>(1) << 45)) return FGE_EINVAL;
    fge_params prm;
    fge_server_config cfg;
    const fge_status st = check_config(p, c, arena_bytes, &prm, &cfg);
    if (st != FGE_OK) return st;
    auto *sx = new (std::nothrow) fge::serve::SimExecutor(sim);
    if (!sx) return FGE_ENOMEM;
    return create_with(prm, cfg, kSimArena, arena_bytes, std::unique_ptr<fge::serve::Executor>(sx),
                       sx, sim.manual == 1, out);
}

int32_t fge_server_sim_step(fge_server *s, int32_t complete, double advance_ms) {
    if (!s || !s->manual || complete < 0 || !(advance_ms >= 0.0)) return FGE_EINVAL;
    std::lock_guard<std::mutex> step(s->step_mu);
    s->sim->step(complete, advance_ms);
    int32_t enqueued = 0;
    for (;;) {
        const Pass r = pass(s);
        if (r == kFatal) return static_cast<int32_t>(s->error);
        if (r != kProgress) break;
        ++enqueued;
    }
    return enqueued;
}

int32_t fge_server_sim_inflight(fge_server *s) {
    if (!s || !s->sim) return FGE_EINVAL;
    return s->sim->outstanding();
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
    r->submit_ms = s->exec->now_ms();
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

fge_status fge_server_cancel(fge_server *s, int64_t id) {
    if (!s) return FGE_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    for (std::deque<Request *> *q : {&s->incoming, &s->pending}) {
        for (auto it = q->begin(); it != q->end(); ++it) {
            if ((*it)->id != id) continue;
            Request *r = *it;
            q->erase(it);
            s->results.push_back(make_result(r, FGE_ECANCELED, s->exec->now_ms()));
            ++s->completed;
            s->stats.completed = s->completed;
            ++s->stats.cancelled;
            s->cv_idle.notify_all();
            delete r;
            return FGE_OK;
        }
    }
    return FGE_EINVAL;   // unknown, already admitted, or completed
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
    if (s->manual) {
        // The caller's thread is the scheduler: complete ticks until everything is done.
        for (;;) {
            {
                std::lock_guard<std::mutex> g(s->mu);
                if (s->completed >= s->submitted) return static_cast<fge_status>(s->error);
            }
            const int32_t inflight = s->sim->outstanding();
            const int32_t r = fge_server_sim_step(s, inflight, 0.0);
            if (r < 0) return static_cast<fge_status>(r);
            if (r == 0 && inflight == 0) return FGE_EINVAL;   // nothing can move (cannot happen)
        }
    }
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
    } else if (s->manual && s->exec) {
        fge_server_drain(s);
    }
    for (fge::serve::Slot &sl : s->slots)
        for (Request *r : sl.finishing) delete r;
    for (Request *r : s->active) delete r;
    for (Request *r : s->pending) delete r;
    for (Request *r : s->incoming) delete r;
    delete s;
}

}  // extern "C"
