// Autotuner (C ABI in include/fge.h): times candidate execution settings of one workload on the
// device and returns the fastest.
//
// The two settings searched change how the work is cut, never what is computed:
//   - strip height of the streaming kernel (the halo is fixed by the two fused sweeps of a fine
//     level; the strip height sets how many output rows share one halo, against how many waves
//     the level offers the machine);
//   - the tile-kernel threshold (fine levels up to this many pixels run on the LDS tile kernel,
//     larger ones on the streaming kernel).
// Each candidate runs once untimed, then `reps` times between two events on the caller's
// stream; the fastest mean wins.
#include <hip/hip_runtime.h>

#include <vector>

#include "fge_internal.h"

namespace {

constexpr int kRows[] = {0, 16, 24, 32, 48, 64, 96};
constexpr int kTileMax[] = {1 << 16, 1 << 18, 1 << 20};

struct Candidate {
    fge_params p;
};

std::vector<Candidate> candidates(const fge_params &base) {
    std::vector<Candidate> out;
    for (int t : kTileMax)
        for (int r : kRows) {
            Candidate c{base};
            c.p.strip_rows = r;
            c.p.tile_max_px = t;
            out.push_back(c);
        }
    return out;
}

// Mean milliseconds of `reps` calls of run() on stream s (after one untimed call).
template <typename Run>
fge_status time_it(Run run, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *ms) {
    fge_status st = run();
    if (st != FGE_OK) return st;
    if (hipEventRecord(e0, s) != hipSuccess) return FGE_EHIP;
    for (int k = 0; k < reps; ++k)
        if ((st = run()) != FGE_OK) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        return FGE_EHIP;
    *ms /= static_cast<float>(reps);
    return FGE_OK;
}

template <typename Run>
fge_status search(const fge_params &base, int reps, void *stream, Run run_with, fge_params *best,
                  fge_tune_entry *entries, int32_t max_entries, int32_t *n_entries) {
    if (reps <= 0) reps = 3;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return FGE_EHIP;
    }
    float best_ms = -1.0f;
    int k = 0;
    fge_status result = FGE_OK;
    const std::vector<Candidate> cands = candidates(base);
    for (size_t idx = 0; idx < cands.size(); ++idx) {
        const Candidate &c = cands[idx];
        float ms = 0.0f;
        const fge_status st = time_it([&] { return run_with(idx, c.p); }, reps, s, e0, e1, &ms);
        if (entries && k < max_entries) entries[k] = fge_tune_entry{c.p.strip_rows, c.p.tile_max_px, ms, st};
        ++k;
        if (st == FGE_EHIP) {   // a failed launch ends the search
            result = st;
            break;
        }
        if (st == FGE_OK && (best_ms < 0.0f || ms < best_ms)) {
            best_ms = ms;
            *best = c.p;
        }
    }
    if (n_entries) *n_entries = k;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result == FGE_OK && best_ms < 0.0f) result = FGE_EUNSUPPORTED;
    return result;
}

const fge_params &resolve(const fge_params *p, fge_params &tmp) {
    if (p) return *p;
    fge_default_params(&tmp);
    return tmp;
}

}  // namespace

extern "C" {

int32_t fge_tune_candidates(void) {
    return static_cast<int32_t>(sizeof(kRows) / sizeof(kRows[0]) * sizeof(kTileMax) / sizeof(kTileMax[0]));
}

size_t fge_tune_workspace_bytes(int32_t H, int32_t W, const fge_params *p) {
    fge_params tmp;
    const fge_params &base = resolve(p, tmp);
    size_t need = 0;
    for (const Candidate &c : candidates(base)) {
        fge::Plan pl;
        if (fge::make_plan(W, H, c.p, &pl, fge::kPlanSingle) != FGE_OK) return 0;
        if (pl.ws_bytes > need) need = pl.ws_bytes;
    }
    return need;
}

fge_status fge_autotune(const void *I, const void *alpha, int32_t H, int32_t W, const fge_params *p,
                        void *F, void *B, void *workspace, size_t workspace_bytes, void *stream,
                        int32_t reps, fge_params *best, fge_tune_entry *entries,
                        int32_t max_entries, int32_t *n_entries) {
    fge_params tmp;
    const fge_params &base = resolve(p, tmp);
    if (!best || reps < 0 || reps > 1000) return FGE_EINVAL;
    fge::Plan pl;
    const fge_status st = fge::make_plan(W, H, base, &pl);
    if (st != FGE_OK) return st;
    if (!I || !alpha || !F || !B) return FGE_EINVAL;
    if (fge::outputs_alias(I, alpha, F, B, W, H, base.storage == FGE_F16 ? 2 : 4, workspace,
                           workspace_bytes))
        return FGE_EINVAL;
    const size_t need = fge_tune_workspace_bytes(H, W, &base);
    if (need > 0 && (!workspace || workspace_bytes < need)) return FGE_EWORKSPACE;
    return search(base, reps, stream,
                  [&](size_t, const fge_params &q) {
                      return fge_estimate_foreground(I, alpha, H, W, &q, F, B, workspace,
                                                     workspace_bytes, stream);
                  },
                  best, entries, max_entries, n_entries);
}

size_t fge_batch_tune_workspace_bytes(int32_t n, const int32_t *H, const int32_t *W,
                                      const fge_params *p) {
    fge_params tmp;
    const fge_params &base = resolve(p, tmp);
    size_t need = 0;
    for (const Candidate &c : candidates(base)) {
        const size_t v = fge_batch_workspace_bytes_for(n, H, W, &c.p);
        if (v == 0) return 0;
        if (v > need) need = v;
    }
    return need;
}

fge_status fge_batch_autotune(int32_t n, const void *const *I, const void *const *alpha,
                              const int32_t *H, const int32_t *W, const fge_params *p,
                              void *const *F, void *const *B, void *workspace,
                              size_t workspace_bytes, void *stream, int32_t reps, fge_params *best,
                              fge_tune_entry *entries, int32_t max_entries, int32_t *n_entries) {
    fge_params tmp;
    const fge_params &base = resolve(p, tmp);
    if (!best || reps < 0 || reps > 1000) return FGE_EINVAL;
    const size_t need = fge_batch_tune_workspace_bytes(n, H, W, &base);
    if (need == 0) return FGE_EINVAL;
    if (!workspace || workspace_bytes < need) return FGE_EWORKSPACE;
    std::vector<fge_batch *> plans;
    fge_status st = FGE_OK;
    for (const Candidate &c : candidates(base)) {
        fge_batch *b = nullptr;
        st = fge_batch_create(n, H, W, &c.p, &b);
        if (st != FGE_OK) break;
        plans.push_back(b);
    }
    if (st == FGE_OK)
        st = search(base, reps, stream,
                    [&](size_t idx, const fge_params &) {
                        return fge_batch_run(plans[idx], I, alpha, F, B, workspace,
                                             workspace_bytes, stream);
                    },
                    best, entries, max_entries, n_entries);
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess && st == FGE_OK) st = FGE_EHIP;
    for (fge_batch *b : plans) fge_batch_destroy(b);
    return st;
}

}  // extern "C"
