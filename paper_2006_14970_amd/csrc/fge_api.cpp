// C ABI of libfge (declared in include/fge.h): argument checks, the launch sequence of
// Algorithm 1's levels on the caller's stream, and optional per-level event timing.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "fge_internal.h"

namespace {

constexpr int32_t kAbiVersion = 9;

struct ProfileRecord {
    int level;          // 0 = finest
    hipEvent_t start, stop;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<ProfileRecord> recs;   // events created in fge_profile_start
    size_t used = 0;
};

Profiler &profiler() {
    static Profiler p;
    return p;
}

// Brackets one launch with events when profiling is on.
struct LaunchTimer {
    ProfileRecord *rec = nullptr;
    hipStream_t s;
    LaunchTimer(int level_from_finest, hipStream_t stream) : s(stream) {
        Profiler &p = profiler();
        std::lock_guard<std::mutex> g(p.mu);
        if (p.on && p.used < p.recs.size()) {
            rec = &p.recs[p.used++];
            rec->level = level_from_finest;
            (void)hipEventRecord(rec->start, s);
        }
    }
    ~LaunchTimer() {
        if (rec) (void)hipEventRecord(rec->stop, s);
    }
};

// The launch sequence of Algorithm 1's levels for one image under `plan`, with the workspace at
// `ws` (plan.ws_bytes bytes, 256-byte aligned), on stream `s`.
fge_status run_single(const fge::Plan &plan, const fge_params &prm, const void *I, const void *alpha,
                      void *F, void *B, char *ws, hipStream_t s) {
    const int n = plan.n;
    if (plan.ng > 0 && !plan.gather_in_coarse) {
        LaunchTimer timer(n, s);   // recorded under index n_levels
        if (fge::launch_gather(plan, I, alpha, fge::pyr_base(plan, ws, F), prm.storage, s))
            return FGE_EHIP;
    }
    if (plan.nc > 0) {
        void *fo, *bo;
        fge::level_state(plan, ws, plan.nc - 1, F, B, &fo, &bo);
        const fge::LevelSrc src = fge::coarse_src(plan, ws, F, I, alpha);
        LaunchTimer timer(n - plan.nc, s);
        const int err = plan.gather_in_coarse
                            ? fge::launch_coarse_gather(plan, src, fo, bo, prm.omega, prm.eps_r, I,
                                                        alpha, fge::pyr_base(plan, ws, F),
                                                        prm.storage, s)
                            : fge::launch_coarse(plan, src, fo, bo, prm.omega, prm.eps_r,
                                                 prm.storage, s);
        if (err) return FGE_EHIP;
    }
    for (int i = plan.nc; i < n; ++i) {
        if (i == plan.pyr_first) {   // the run of tile levels in one launch
            LaunchTimer timer(n - 1 - plan.pyr_last, s);   // recorded under the run's last level
            if (fge::launch_pyramid(plan, ws, I, alpha, F, B, prm.omega, prm.eps_r, prm.storage, s))
                return FGE_EHIP;
            i = plan.pyr_last;
            continue;
        }
        const fge::LevelIO io = fge::level_io(plan, ws, i, I, alpha, F, B, prm.omega, prm.eps_r);
        LaunchTimer timer(n - 1 - i, s);
        int err = 0;
        switch (plan.kind[i]) {
            case fge::kKindStream: err = fge::launch_fine_fused(io, prm.strip_rows, prm.storage, s); break;
            case fge::kKindTile: err = fge::launch_fine_tile(io, prm.storage, s); break;
            default: err = fge::launch_naive_level(io, plan.lv[i].iters, prm.storage, s); break;
        }
        if (err) return FGE_EHIP;
    }
    return FGE_OK;
}

// ---- the allocation-free single-image call -----------------------------------------------
//
// fge_estimate_foreground_noalloc keeps the single-image workspace in this file-scope device
// array instead of a caller buffer.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with hipGetSymbolAddress (each device
// holds its own copy of the array) and only that address is passed to kernels.
constexpr size_t kScratchBytes = FGE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

struct ScratchTable {
    std::mutex mu;
    void *ptr[kMaxDevices] = {};
};

ScratchTable &scratch_table() {
    static ScratchTable t;
    return t;
}

// The device address of `scratch` on the current device (looked up on the first call there).
fge_status scratch_on_current_device(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FGE_EHIP;
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FGE_EHIP;
        t.ptr[dev] = p;
    }
    *out = static_cast<char *>(t.ptr[dev]);
    return FGE_OK;
}

const fge_params &resolve(const fge_params *p, fge_params &tmp) {
    if (p) return *p;
    fge_default_params(&tmp);
    return tmp;
}

}  // namespace

extern "C" {

void fge_default_params(fge_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->size = sizeof(fge_params);
    p->omega = 0.1f;
    p->eps_r = 5e-3f;
    p->small_size = 32;
    p->iters_small = 10;
    p->iters_big = 2;
    p->storage = FGE_F32;
    p->order = FGE_REDBLACK;
    p->kernel = FGE_KERNEL_AUTO;
    p->strip_rows = 0;
    p->coarse_max_px = 0;
    p->tile_max_px = 0;
}

const char *fge_status_string(int status) {
    switch (status) {
        case FGE_OK: return "FGE_OK";
        case FGE_EINVAL: return "FGE_EINVAL: invalid argument";
        case FGE_ENOMEM: return "FGE_ENOMEM: host allocation failed";
        case FGE_EHIP: return "FGE_EHIP: HIP runtime or launch error";
        case FGE_EUNSUPPORTED: return "FGE_EUNSUPPORTED: not implemented for these parameters";
        case FGE_EWORKSPACE: return "FGE_EWORKSPACE: workspace missing or too small";
        case FGE_EBUDGET: return "FGE_EBUDGET: request larger than the server budget or arena";
        case FGE_ECANCELED: return "FGE_ECANCELED: request cancelled before admission";
        default: return "unknown fge status";
    }
}

int32_t fge_version(void) { return kAbiVersion; }

int32_t fge_num_levels(int32_t H, int32_t W) {
    if (W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return 0;
    return fge::num_levels(W, H);
}

int32_t fge_level_size(int32_t full, int32_t level, int32_t n_levels) {
    if (full < 1 || full > fge::kMaxSide || n_levels < 1 || n_levels > fge::kMaxLevels ||
        level < 1 || level > n_levels)
        return 0;
    return fge::level_size(full, level, n_levels);
}

fge_status fge_plan(int32_t H, int32_t W, const fge_params *p, int32_t max_levels, int32_t *w_out,
                    int32_t *h_out, int32_t *iters_out, int32_t *n_levels_out,
                    int32_t *n_coarse_out) {
    fge_params tmp;
    fge::Plan plan;
    const fge_status st = fge::make_plan(W, H, resolve(p, tmp), &plan);
    if (st != FGE_OK) return st;
    if (max_levels < plan.n) return FGE_EINVAL;
    for (int i = 0; i < plan.n; ++i) {
        if (w_out) w_out[i] = plan.lv[i].w;
        if (h_out) h_out[i] = plan.lv[i].h;
        if (iters_out) iters_out[i] = plan.lv[i].iters;
    }
    if (n_levels_out) *n_levels_out = plan.n;
    if (n_coarse_out) *n_coarse_out = plan.nc;
    return FGE_OK;
}

size_t fge_workspace_bytes(int32_t H, int32_t W, const fge_params *p) {
    fge_params tmp;
    fge::Plan plan;
    const fge_params &prm = resolve(p, tmp);
    if (fge::make_plan(W, H, prm, &plan, fge::kPlanSingle) != FGE_OK) return 0;
    if (prm.order == FGE_JACOBI) return fge::converge_workspace_bytes(W, H, prm);
    return plan.ws_bytes;
}

fge_status fge_estimate_foreground(const void *I, const void *alpha, int32_t H, int32_t W,
                                   const fge_params *p, void *F, void *B, void *workspace,
                                   size_t workspace_bytes, void *stream) {
    fge_params tmp;
    const fge_params &prm = resolve(p, tmp);
    fge::Plan plan;
    const fge_status st = fge::make_plan(W, H, prm, &plan, fge::kPlanSingle);
    if (st != FGE_OK) return st;
    if (!I || !alpha || !F || !B) return FGE_EINVAL;
    if (fge::outputs_alias(I, alpha, F, B, W, H, plan.elem, workspace, workspace_bytes))
        return FGE_EINVAL;
    if (prm.order == FGE_JACOBI)   // fixed counts on the per-level Jacobi kernels
        return fge::estimate_converge(I, alpha, W, H, prm, -1.0, 0, F, B, nullptr, workspace,
                                      workspace_bytes, stream);
    if (plan.ws_bytes > 0 && (!workspace || workspace_bytes < plan.ws_bytes)) return FGE_EWORKSPACE;
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255)) return FGE_EWORKSPACE;

    return run_single(plan, prm, I, alpha, F, B, static_cast<char *>(workspace),
                      static_cast<hipStream_t>(stream));
}

fge_status fge_estimate_foreground_noalloc(const void *I, const void *alpha, int32_t H, int32_t W,
                                           const fge_params *p, void *F, void *B, void *stream) {
    fge_params tmp;
    const fge_params &prm = resolve(p, tmp);
    fge::Plan plan;
    const fge_status st = fge::make_plan(W, H, prm, &plan, fge::kPlanSingle);
    if (st != FGE_OK) return st;
    if (prm.order == FGE_JACOBI) return FGE_EUNSUPPORTED;   // the per-level path's workspace
    if (!I || !alpha || !F || !B) return FGE_EINVAL;
    if (plan.ws_bytes > kScratchBytes) return FGE_EWORKSPACE;
    char *ws = nullptr;
    const fge_status sst = scratch_on_current_device(&ws);
    if (sst != FGE_OK) return sst;
    if (fge::outputs_alias(I, alpha, F, B, W, H, plan.elem, ws, plan.ws_bytes)) return FGE_EINVAL;
    return run_single(plan, prm, I, alpha, F, B, ws, static_cast<hipStream_t>(stream));
}

fge_status fge_profile_start(int32_t capacity) {
    if (capacity < 1 || capacity > (1 << 20)) return FGE_EINVAL;
    Profiler &p = profiler();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto &r : p.recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    p.recs.clear();
    p.used = 0;
    p.recs.resize(capacity);
    for (auto &r : p.recs) {
        if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess)
            return FGE_EHIP;
    }
    p.on = true;
    return FGE_OK;
}

fge_status fge_profile_stop(double *level_ms, int32_t *level_launches, int32_t max_levels) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = false;
    for (int i = 0; i < max_levels; ++i) {
        if (level_ms) level_ms[i] = 0.0;
        if (level_launches) level_launches[i] = 0;
    }
    fge_status st = FGE_OK;
    for (size_t k = 0; k < p.used; ++k) {
        ProfileRecord &r = p.recs[k];
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            st = FGE_EHIP;
            continue;
        }
        if (r.level >= 0 && r.level < max_levels) {
            if (level_ms) level_ms[r.level] += ms;
            if (level_launches) level_launches[r.level] += 1;
        }
    }
    for (auto &r : p.recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    p.recs.clear();
    p.used = 0;
    return st;
}

}  // extern "C"
