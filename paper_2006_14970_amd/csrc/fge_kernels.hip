// HIP kernels (gfx950) for multi-level foreground estimation, arXiv 2006.14970, Algorithm 1.
//
// Kernel families, all computing in float32 and storing in T (float or _Float16):
//
//  coarse_kernel   One workgroup runs the low-resolution levels (by default those of at most
//                  1024 px, plus every level whose sweep count is not 2) entirely in LDS,
//                  including their 10 sweeps, then writes the last of them to memory.
//                  coarse_gather_kernel runs it in workgroup 0 while the rest of the launch copies
//                  the compact inputs of the later levels (single image).
//
//  tile_kernel     One level, one workgroup per 32x32 output tile plus a 4-pixel ring in LDS.
//                  pyramid_kernel runs a run of consecutive tile levels in one launch, each
//                  workgroup computing exactly the lower-level regions its output tile needs.
//
//  fine_kernel     One launch per large fine level.  Each wave owns a strip of 128 columns (a
//                  pair of adjacent pixels per lane, so every lane has exactly one pixel of each
//                  colour) and streams down its rows: for every new row it gathers I and alpha
//                  (nearest), upsamples F and B from the previous level, and runs all four
//                  red-black half-sweeps of the level's two sweeps on an eight-row register
//                  window (temporal blocking).  Horizontal neighbours cross lanes with DPP;
//                  nothing goes through LDS.  A half-sweep invalidates one ring at the strip
//                  edge, so strips overlap by 4 rows/columns of halo that are computed but not
//                  stored.  One HBM round trip per level.
//
//  batch kernels   Persistent versions of the tile and streaming kernels pulling (level, tile or
//                  strip) items from a work counter, one coarse workgroup per image, a batched
//                  gather.
//
//  naive kernels   Debug path: one launch per upsample and per half-sweep, in place.
//
// Per-pixel update (eq. 9 in Sherman-Morrison form).  With the four clamped neighbours j,
// s_j = eps + omega |a_i - a_j|, S = sum s_j, Fbar = sum s_j F_j / S, Bbar likewise, the 2x2
// system (U U^T + S Id) g = U I + S [Fbar, Bbar] has the solution
//     g = [Fbar, Bbar] + U (I - U^T [Fbar, Bbar]) / (S + |U|^2),   U = [a, 1 - a],
// which needs two reciprocals per pixel that are shared by the three channels, and is well
// conditioned (S + |U|^2 >= 0.5).  The result is clamped to [0, 1] (Algorithm 1).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fge_internal.h"

namespace fge {
namespace {

template <typename T>
__device__ __forceinline__ float ldf(const T *p) {
    return static_cast<float>(*p);
}

template <typename T>
__device__ __forceinline__ void stf(T *p, float v) {
    *p = static_cast<T>(v);
}

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

// v rounded to the storage type T and back (the value a store and a reload would give).
template <typename T>
__device__ __forceinline__ float round_to(float v) {
    return static_cast<float>(static_cast<T>(v));
}

// Reciprocal with v_rcp_f32 (1 ulp); its arguments here are in [0.02, 4].
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Makes a value that is the same in every lane of the wave visible as such to the compiler, so
// that branches on it are scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for every outstanding
// global load of the thread, which would serialise the prefetches issued before a barrier.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Lane i receives v from lane i-1; lane 0 keeps `self` (DPP wave_shr:1, disabled lanes keep old).
__device__ __forceinline__ float from_left(float v, float self) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(self), __float_as_int(v),
                                                      0x138, 0xF, 0xF, false));
}

// Lane i receives v from lane i+1; lane 63 keeps `self` (DPP wave_shl:1).
__device__ __forceinline__ float from_right(float v, float self) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(self), __float_as_int(v),
                                                      0x130, 0xF, 0xF, false));
}

// floor(num / den) for 0 <= num < 2^30 and 1 <= den <= 32767 with a quotient below 32768 (every
// nearest-neighbour map and index split here).  gfx950 has no integer divide; the float estimate
// num * rcp(den) is within 0.01 of num / den (input rounding 2^-24 and rcp 1 ulp, times a
// quotient below 2^15), so one correction step each way makes it exact.  rden = rcp(den).
__device__ __forceinline__ int fdiv(int num, int den, float rden) {
    int q = static_cast<int>(static_cast<float>(num) * rden);
    const int r = num - q * den;
    q += r < 0 ? -1 : (r >= den ? 1 : 0);
    return q;
}

__device__ __forceinline__ float weight(float a, float b, float omega, float eps) {
    return fmaf(omega, fabsf(a - b), eps);
}

// ------------------------------------------------------------------------------------------
// Coarse kernel: levels [0, nc) in LDS.
// ------------------------------------------------------------------------------------------


// Pixel pairs (2j, 2j+1) of row y owned by one thread: thread t owns pairs t and t + 1024.
struct CoarsePair {
    int p0;          // LDS index of the pair's first pixel (y * w + 2j)
    int x0, y;
    bool valid0, valid1;
};

template <typename T>
__device__ __forceinline__ void coarse_gather_inputs(const CoarseArgs &args, int l, int w, int h,
                                                     const CoarsePair (&pr)[kCoarsePairsPerThread],
                                                     float (&ni)[kCoarsePairsPerThread][2][3],
                                                     float (&na)[kCoarsePairsPerThread][2]) {
    const T *I = static_cast<const T *>(args.src.I[l]);
    const T *A = static_cast<const T *>(args.src.A[l]);
    const int W = args.src.W[l], H = args.src.H[l];
    const size_t planeI = static_cast<size_t>(W) * H;
    const bool same = W == w && H == h;   // a compact copy of the level: identity map
    const float rw = rcp(static_cast<float>(w)), rh = rcp(static_cast<float>(h));
#pragma unroll
    for (int k = 0; k < kCoarsePairsPerThread; ++k) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool ok = s == 0 ? pr[k].valid0 : pr[k].valid1;
            const int x = ok ? pr[k].x0 + s : 0, y = ok ? pr[k].y : 0;
            const size_t src = same ? static_cast<size_t>(y) * W + x
                                    : static_cast<size_t>(fdiv(y * H, h, rh)) * W + fdiv(x * W, w, rw);
            na[k][s] = ldf(A + src);
#pragma unroll
            for (int c = 0; c < 3; ++c) ni[k][s][c] = ldf(I + c * planeI + src);
        }
    }
}

__device__ __forceinline__ void coarse_pairs(int tid, int w, int h,
                                             CoarsePair (&pr)[kCoarsePairsPerThread]) {
    const int pw = (w + 1) >> 1;
    const float rpw = rcp(static_cast<float>(pw));
#pragma unroll
    for (int k = 0; k < kCoarsePairsPerThread; ++k) {
        const int q = tid + k * kCoarseThreads;
        const int y = fdiv(q, pw, rpw);
        const int j = q - y * pw;
        pr[k].y = y;
        pr[k].x0 = 2 * j;
        pr[k].p0 = y * w + 2 * j;
        pr[k].valid0 = y < h;
        pr[k].valid1 = y < h && 2 * j + 1 < w;
    }
}

// Per pixel two float4 records: (F0, F1, F2, alpha) and (B0, B1, B2, unused).
struct CoarseLds {
    float4 FA[kCoarseMaxPx];
    float4 B[kCoarseMaxPx];
};

// The convergence form on the coarse block (CONV): a level runs passes of two sweeps until a pass
// changes the level's energy by at most tol times its value before the pass, or max_passes passes
// have run; the passes a level ran go to counts[l].  red: 2 * (kCoarseThreads / 64) doubles of
// LDS for the energy's per-wave sums.
struct CoarseConv {
    double tol;
    int max_passes;
    int *counts;
    double *red;
};

template <typename T, bool CONV = false>
__device__ __forceinline__ void coarse_body(const CoarseArgs &args, CoarseLds &lds,
                                            const CoarseConv &cv = CoarseConv{}) {
    float4 *sFA = lds.FA;
    float4 *sB = lds.B;

    const int tid = threadIdx.x;
    const float omega = args.omega, eps = args.eps;

    const int wave_q0 = uniform(tid & ~63);   // first pair index of this wave in slot 0
    CoarsePair pr[kCoarsePairsPerThread];
    float iv[kCoarsePairsPerThread][2][3], av[kCoarsePairsPerThread][2];
    float ni[kCoarsePairsPerThread][2][3], na[kCoarsePairsPerThread][2];
    coarse_pairs(tid, args.lw[0], args.lh[0], pr);
    coarse_gather_inputs<T>(args, 0, args.lw[0], args.lh[0], pr, ni, na);

    // A pair slot k is live in a wave when some lane of the wave owns a pair of the level there;
    // the LDS stores, the per-level constants and the sweeps of dead slots are skipped as a
    // whole (a uniform test).  (Skipping the resize reads and the input gathers too would spill.)
    int wp = 1, hp = 1;
    for (int l = 0; l < args.nc; ++l) {
        const int w = args.lw[l], h = args.lh[l], iters = args.lit[l];
        const int npairs = ((w + 1) >> 1) * h;
        auto live = [&](int k) { return k * kCoarseThreads + wave_q0 < npairs; };
#pragma unroll
        for (int k = 0; k < kCoarsePairsPerThread; ++k)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                av[k][s] = na[k][s];
#pragma unroll
                for (int c = 0; c < 3; ++c) iv[k][s][c] = ni[k][s][c];
            }
        // Resize F and B from the previous level (the 1x1 zero start before level 0): gather
        // into registers, then overwrite LDS with the new level.
        float4 rf[kCoarsePairsPerThread][2], rb[kCoarsePairsPerThread][2];
        const float rw = rcp(static_cast<float>(w)), rh = rcp(static_cast<float>(h));
#pragma unroll
        for (int k = 0; k < kCoarsePairsPerThread; ++k) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rf[k][s] = make_float4(0.f, 0.f, 0.f, av[k][s]);
                rb[k][s] = make_float4(0.f, 0.f, 0.f, 0.f);
                const bool ok = (s == 0 ? pr[k].valid0 : pr[k].valid1) && l > 0;
                const int q = ok ? fdiv(pr[k].y * hp, h, rh) * wp + fdiv((pr[k].x0 + s) * wp, w, rw) : 0;
                const float4 f = sFA[q];
                const float4 g = sB[q];
                if (ok) {
                    rf[k][s] = make_float4(f.x, f.y, f.z, av[k][s]);
                    rb[k][s] = g;
                }
            }
        }
        lds_sync();
#pragma unroll
        for (int k = 0; k < kCoarsePairsPerThread; ++k) {
            if (!live(k)) continue;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bool ok = s == 0 ? pr[k].valid0 : pr[k].valid1;
                if (ok) {
                    sFA[pr[k].p0 + s] = rf[k][s];
                    sB[pr[k].p0 + s] = rb[k][s];
                }
            }
        }
        // Start the next level's input gather now; it completes during this level's sweeps.
        CoarsePair nx[kCoarsePairsPerThread];
        if (l + 1 < args.nc) {
            coarse_pairs(tid, args.lw[l + 1], args.lh[l + 1], nx);
            coarse_gather_inputs<T>(args, l + 1, args.lw[l + 1], args.lh[l + 1], nx, ni, na);
        }
        lds_sync();

        // Per-pixel constants of this level, stored by colour: entry [k][c] describes the pixel
        // of pair k updated in half-sweep c, i.e. column x0 + ((y + c) & 1).
        int cpix[kCoarsePairsPerThread][2], cnb[kCoarsePairsPerThread][2][4];
        bool cok[kCoarsePairsPerThread][2];
        float cw[kCoarsePairsPerThread][2][4], cka[kCoarsePairsPerThread][2], ckb[kCoarsePairsPerThread][2];
        float ca[kCoarsePairsPerThread][2], ci[kCoarsePairsPerThread][2][3];
#pragma unroll
        for (int k = 0; k < kCoarsePairsPerThread; ++k) {
            if (!live(k)) continue;
            int tnb[2][4];
            float tw[2][4], tka[2], tkb[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int x = min(pr[k].x0 + s, w - 1), y = min(pr[k].y, h - 1);
                const int i = y * w + x;
                tnb[s][0] = x > 0 ? i - 1 : i;
                tnb[s][1] = x < w - 1 ? i + 1 : i;
                tnb[s][2] = y > 0 ? i - w : i;
                tnb[s][3] = y < h - 1 ? i + w : i;
                const float a = av[k][s];
                float sj[4], S = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sj[j] = weight(a, sFA[tnb[s][j]].w, omega, eps);
                    S += sj[j];
                }
                const float iS = rcp(S), b = 1.0f - a;
                const float kk = rcp(S + fmaf(a, a, b * b));
#pragma unroll
                for (int j = 0; j < 4; ++j) tw[s][j] = sj[j] * iS;
                tka[s] = a * kk;
                tkb[s] = b * kk;
            }
            const bool odd = pr[k].y & 1;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // pixel slot updated in half-sweep c: c for even rows, 1 - c for odd rows
                const bool hi = odd ? (c == 0) : (c == 1);
                cpix[k][c] = pr[k].p0 + (hi ? 1 : 0);
                cok[k][c] = hi ? pr[k].valid1 : pr[k].valid0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    cnb[k][c][j] = hi ? tnb[1][j] : tnb[0][j];
                    cw[k][c][j] = hi ? tw[1][j] : tw[0][j];
                }
                cka[k][c] = hi ? tka[1] : tka[0];
                ckb[k][c] = hi ? tkb[1] : tkb[0];
                ca[k][c] = hi ? av[k][1] : av[k][0];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) ci[k][c][ch] = hi ? iv[k][1][ch] : iv[k][0][ch];
            }
        }

        // Sweeps: in half-sweep c every pair updates its pixel of colour c.  Pair slots that no
        // lane of the wave uses are skipped as a whole (a uniform test); inside a slot the
        // reads and the arithmetic are unconditional (indices are clamped), only the store is
        // guarded, so the slot's LDS reads are all in flight together.
        auto update = [&](int k, int c) {
                        float fb[3] = {0.f, 0.f, 0.f}, bb[3] = {0.f, 0.f, 0.f};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float wj = cw[k][c][j];
                            const float4 f = sFA[cnb[k][c][j]];
                            const float4 g = sB[cnb[k][c][j]];
                            fb[0] = fmaf(wj, f.x, fb[0]);
                            fb[1] = fmaf(wj, f.y, fb[1]);
                            fb[2] = fmaf(wj, f.z, fb[2]);
                            bb[0] = fmaf(wj, g.x, bb[0]);
                            bb[1] = fmaf(wj, g.y, bb[1]);
                            bb[2] = fmaf(wj, g.z, bb[2]);
                        }
                        const float a = ca[k][c], b = 1.0f - a;
                        float fo[3], bo[3];
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) {
                            const float r = ci[k][c][ch] - a * fb[ch] - b * bb[ch];
                            fo[ch] = clamp01(fmaf(cka[k][c], r, fb[ch]));
                            bo[ch] = clamp01(fmaf(ckb[k][c], r, bb[ch]));
                        }
                        if (cok[k][c]) {
                            sFA[cpix[k][c]] = make_float4(fo[0], fo[1], fo[2], a);
                            sB[cpix[k][c]] = make_float4(bo[0], bo[1], bo[2], 0.0f);
                        }
        };
        // n_it sweeps of the level; every thread leaves through a workgroup barrier.
        auto sweeps = [&](int n_it) {
            if (npairs <= 64) {
                // The whole level is slot 0 of wave 0.  A wave's LDS operations execute in order,
                // so its half-sweeps need no workgroup barrier, only an ordering point for the
                // compiler; the other waves wait at the barrier that ends the level.
                if (uniform(tid >> 6) == 0) {
                    for (int it = 0; it < n_it; ++it) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            update(0, c);
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
                        }
                    }
                }
                lds_sync();
            } else {
                for (int it = 0; it < n_it; ++it) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
#pragma unroll
                        for (int k = 0; k < kCoarsePairsPerThread; ++k)
                            if (live(k)) update(k, c);
                        lds_sync();
                    }
                }
            }
        };
        if constexpr (!CONV) {
            sweeps(iters);
        } else {
            // The level's energy (the data term of every pixel plus, for each pixel, its right
            // and lower edge, so every edge once), each term in float64 from the stored values:
            // per thread, then per wave (butterfly sums, equal in every lane), then over the
            // waves in a fixed order by every thread, so the stop decision is the same
            // everywhere.  Called by all threads after a barrier; the barrier inside separates
            // the per-wave stores from the reads, and the next call's stores come after the
            // sweeps' closing barrier.
            auto energy = [&]() {
                double data = 0.0, smooth = 0.0;
#pragma unroll
                for (int k = 0; k < kCoarsePairsPerThread; ++k) {
                    if (!live(k)) continue;
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        if (!(s == 0 ? pr[k].valid0 : pr[k].valid1)) continue;
                        const int i = pr[k].p0 + s, x = pr[k].x0 + s, y = pr[k].y;
                        const float4 f = sFA[i], g = sB[i];
                        const double a = av[k][s], b = 1.0 - a;
                        const double fv[3] = {f.x, f.y, f.z}, bv[3] = {g.x, g.y, g.z};
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) {
                            const double r = a * fv[ch] + b * bv[ch] - static_cast<double>(iv[k][s][ch]);
                            data += r * r;
                        }
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            if (e == 0 ? x + 1 >= w : y + 1 >= h) continue;
                            const int j = e == 0 ? i + 1 : i + w;
                            const float4 fj = sFA[j], gj = sB[j];
                            const double wgt = static_cast<double>(eps) +
                                               static_cast<double>(omega) * fabs(a - static_cast<double>(fj.w));
                            const double df[3] = {fv[0] - fj.x, fv[1] - fj.y, fv[2] - fj.z};
                            const double db[3] = {bv[0] - gj.x, bv[1] - gj.y, bv[2] - gj.z};
                            double d = 0.0;
#pragma unroll
                            for (int ch = 0; ch < 3; ++ch) d += df[ch] * df[ch] + db[ch] * db[ch];
                            smooth += wgt * d;
                        }
                    }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    data += __shfl_xor(data, off);
                    smooth += __shfl_xor(smooth, off);
                }
                constexpr int kWaves = kCoarseThreads / 64;
                if ((tid & 63) == 0) {
                    cv.red[tid >> 6] = data;
                    cv.red[kWaves + (tid >> 6)] = smooth;
                }
                lds_sync();
                double D = 0.0, Sm = 0.0;
#pragma unroll
                for (int q = 0; q < kWaves; ++q) {
                    D += cv.red[q];
                    Sm += cv.red[kWaves + q];
                }
                return D + Sm;
            };
            double e_prev = energy();
            int k = 0;
            for (;;) {
                sweeps(2);
                const double e = energy();
                ++k;
                const bool stop = fabs(e_prev - e) <= cv.tol * e_prev || k >= cv.max_passes;
                if (uniform(stop ? 1 : 0)) break;
                e_prev = e;
            }
            if (tid == 0) cv.counts[l] = k;
        }
        if (l + 1 < args.nc) {
#pragma unroll
            for (int k = 0; k < kCoarsePairsPerThread; ++k) pr[k] = nx[k];
        }
        wp = w;
        hp = h;
    }

    // Write the last coarse level.
    T *Fo = static_cast<T *>(args.Fo);
    T *Bo = static_cast<T *>(args.Bo);
    const int n = wp * hp;
    for (int p = tid; p < n; p += kCoarseThreads) {
        const float4 f = sFA[p], g = sB[p];
        stf(Fo + p, f.x);
        stf(Fo + n + p, f.y);
        stf(Fo + 2 * static_cast<size_t>(n) + p, f.z);
        stf(Bo + p, g.x);
        stf(Bo + n + p, g.y);
        stf(Bo + 2 * static_cast<size_t>(n) + p, g.z);
    }
}

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void coarse_kernel(CoarseArgs args) {
    __shared__ CoarseLds lds;
    coarse_body<T>(args, lds);
}

// Batch: workgroup b runs the coarse block of image b.
// The coarse levels in the convergence form (float32 state and inputs).
__global__ __launch_bounds__(kCoarseThreads) void coarse_conv_kernel(CoarseArgs args, double tol,
                                                                     int max_passes, int *counts) {
    __shared__ CoarseLds lds;
    __shared__ double red[2 * (kCoarseThreads / 64)];
    coarse_body<float, true>(args, lds, CoarseConv{tol, max_passes, counts, red});
}

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void coarse_batch_kernel(const CoarseArgs *descs) {
    __shared__ CoarseLds lds;
    coarse_body<T>(descs[blockIdx.x], lds);
}

// ------------------------------------------------------------------------------------------
// Tile kernel: one fine level, one workgroup per 32x32 output tile, state in LDS.
// ------------------------------------------------------------------------------------------
//
// The workgroup loads its tile plus a ring of kTileHalo pixels (clamped to the image) in one
// shot -- alpha, F and B into LDS, I into registers -- runs the level's red-black half-sweeps
// with neighbours clamped to the loaded region, and stores the core.  Where the region edge is
// the image border the clamp is exactly Algorithm 1's; elsewhere the ring absorbs the stale
// neighbours (one ring per half-sweep).  For mid-size levels this replaces the streaming
// kernel's per-row pipeline fill by a single memory round trip.

constexpr int kTileCore = 32;
constexpr int kTileHalo = 4;                      // = half-sweeps of a 2-sweep level
constexpr int kTileSide = kTileCore + 2 * kTileHalo;
constexpr int kTilePx = kTileSide * kTileSide;
constexpr int kTileThreads = 512;
constexpr int kTilePairs = (kTileSide / 2) * kTileSide;
constexpr int kTilePairsPerThread = (kTilePairs + kTileThreads - 1) / kTileThreads;


struct TileLds {
    float4 FA[kTilePx];   // (F0, F1, F2, alpha)
    float4 B[kTilePx];    // (B0, B1, B2, unused)
};

// Records of a region in LDS, split by red-black colour: pixel (x, y) of the region (relative
// coordinates, global colour g) at g * kTileHalf + y * pw + x / 2, pw = ceil(width / 2).  The
// pixels one half-sweep updates then sit at consecutive records for consecutive pairs, and so do
// the neighbours they read (all of the other colour): 16-byte accesses without bank conflicts.
constexpr int kTileHalf = kTilePx / 2;   // >= pw * height for every region (width, height <= 40)
__device__ __forceinline__ int tile_slot(int x, int y, int colour, int pw) {
    return colour * kTileHalf + y * pw + (x >> 1);
}

// The part of a level one tile pass computes: region [rx0, rx0 + rw) x [ry0, ry0 + rh) of the
// level (the core plus a ring of up to kTileHalo pixels, clamped to the image), and the core
// [cx0, cx1) x [cy0, cy1) whose values come out exact.
struct TileRegion {
    int rx0, ry0, rw, rh;
    int cx0, cx1, cy0, cy1;
};

__device__ __forceinline__ TileRegion tile_region(int cx0, int cx1, int cy0, int cy1, int w, int h) {
    TileRegion R;
    R.cx0 = cx0;
    R.cx1 = cx1;
    R.cy0 = cy0;
    R.cy1 = cy1;
    R.rx0 = max(0, cx0 - kTileHalo);
    R.ry0 = max(0, cy0 - kTileHalo);
    R.rw = min(w, cx1 + kTileHalo) - R.rx0;
    R.rh = min(h, cy1 + kTileHalo) - R.ry0;
    return R;
}

// Where a tile pass takes the previous level's F and B: global memory (the stored level), or
// the region of the previous level another pass of the same workgroup left in LDS.
struct TilePrev {
    const void *Fp, *Bp;            // global: 3 planes of wp x hp each
    const float4 *sFA, *sB;         // LDS: the previous level's region records (tile_slot)
    int rx0, ry0, pw;               // LDS: that region's origin and half width, rounded up
    int wp, hp;
};

// The level inputs of the pixels one thread owns in a tile pass over region R: pair
// q = tid + k * threads covers region columns (2j, 2j+1) of region row y.
struct TileInput {
    float a[kTilePairsPerThread][2];
    float iv[kTilePairsPerThread][2][3];
};

// Issue the gathers of alpha and I of region R (they complete in the background: nothing here
// waits for them).
template <typename T>
__device__ __forceinline__ void tile_fetch(const T *I, const T *A, int W, int H, int w, int h,
                                           const TileRegion &R, TileInput &in) {
    const size_t planeI = static_cast<size_t>(W) * H;
    const int pw = (R.rw + 1) >> 1;
    const int npairs = pw * R.rh;
    const float rpw = rcp(static_cast<float>(pw));
    const float rcw = rcp(static_cast<float>(w)), rch = rcp(static_cast<float>(h));
    const bool same = W == w && H == h;   // compact copy or the full-size level
#pragma unroll
    for (int k = 0; k < kTilePairsPerThread; ++k) {
        const int q = threadIdx.x + k * kTileThreads;
        const int y = fdiv(q, pw, rpw);
        const int x = 2 * (q - y * pw);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool ok = q < npairs && x + s < R.rw;
            const int gx = R.rx0 + (ok ? x + s : 0), gy = R.ry0 + (ok ? y : 0);
            const size_t src = same ? static_cast<size_t>(gy) * w + gx
                                    : static_cast<size_t>(fdiv(gy * H, h, rch)) * W +
                                          fdiv(gx * W, w, rcw);
            in.a[k][s] = ldf(A + src);
#pragma unroll
            for (int c = 0; c < 3; ++c) in.iv[k][s][c] = ldf(I + c * planeI + src);
        }
    }
}

// One level of a tile pass over region R, with its inputs fetched (tile_fetch): load F and B
// of the region (alpha, F and B into LDS), run the level's red-black half-sweeps with
// neighbours clamped to the region, and store the core to Fo, Bo when they are given.  Where
// the region edge is the image border the clamp is exactly Algorithm 1's; elsewhere the ring
// absorbs the stale neighbours (one ring per half-sweep).  Previous-level values taken from LDS
// are rounded to the storage type first, as they would have been on their way through memory,
// so the result does not depend on the path.
//
// EN (the energy kernel): before sweeping, the workgroup also reduces the energy of the state it
// loaded over its core pixels (data term, right and lower edge of each, so every edge of the
// level once; each pixel's terms in float32, summed in float64) and thread 0 writes it to
// epart[5 * unit] (then zeros; the layout of fge_energy's partial sums).  ered: kTileThreads / 64
// doubles of LDS.
template <typename T, bool PREV_LDS, bool EN = false, bool JAC = false>
__device__ __forceinline__ void tile_level(const TileInput &in, int w, int h, const TilePrev &pv,
                                           const TileRegion &R, float4 *sFA, float4 *sB,
                                           float omega, float eps, T *Fo, T *Bo,
                                           double *epart = nullptr, int unit = 0,
                                           double *ered = nullptr) {
    const T *Fp = static_cast<const T *>(pv.Fp);
    const T *Bp = static_cast<const T *>(pv.Bp);
    const size_t planeP = static_cast<size_t>(pv.wp) * pv.hp;
    const int tid = threadIdx.x;

    const int rx0 = R.rx0, ry0 = R.ry0, rw = R.rw, rh = R.rh;
    const int pw = (rw + 1) >> 1;
    const int npairs = pw * rh;
    const float rpw = rcp(static_cast<float>(pw));
    const float rcw = rcp(static_cast<float>(w)), rch = rcp(static_cast<float>(h));

    // Owned pairs as in tile_fetch.  All global gathers are issued before any LDS store, so
    // they are in flight together.
    int qy[kTilePairsPerThread], qx[kTilePairsPerThread];
    bool qv0[kTilePairsPerThread], qv1[kTilePairsPerThread];
    float4 lf[kTilePairsPerThread][2], lb[kTilePairsPerThread][2];
#pragma unroll
    for (int k = 0; k < kTilePairsPerThread; ++k) {
        const int q = tid + k * kTileThreads;
        const int y = fdiv(q, pw, rpw);
        qy[k] = y;
        qx[k] = 2 * (q - y * pw);
        qv0[k] = q < npairs;
        qv1[k] = q < npairs && qx[k] + 1 < rw;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool ok = s ? qv1[k] : qv0[k];
            const int gx = rx0 + (ok ? qx[k] + s : 0), gy = ry0 + (ok ? y : 0);
            const int px = fdiv(gx * pv.wp, w, rcw), py = fdiv(gy * pv.hp, h, rch);
            const float a = in.a[k][s];
            if constexpr (PREV_LDS) {
                const int li = tile_slot(px - pv.rx0, py - pv.ry0, (px + py) & 1, pv.pw);
                const float4 f = pv.sFA[ok ? li : 0], g = pv.sB[ok ? li : 0];
                lf[k][s] = make_float4(round_to<T>(f.x), round_to<T>(f.y), round_to<T>(f.z), a);
                lb[k][s] = make_float4(round_to<T>(g.x), round_to<T>(g.y), round_to<T>(g.z), 0.0f);
            } else {
                const size_t prv = static_cast<size_t>(py) * pv.wp + px;
                lf[k][s] = make_float4(ldf(Fp + prv), ldf(Fp + planeP + prv), ldf(Fp + 2 * planeP + prv), a);
                lb[k][s] = make_float4(ldf(Bp + prv), ldf(Bp + planeP + prv), ldf(Bp + 2 * planeP + prv), 0.0f);
            }
        }
    }
    // (From LDS the previous region and this one are different buffers: no barrier between.)
#pragma unroll
    for (int k = 0; k < kTilePairsPerThread; ++k)
#pragma unroll
        for (int s = 0; s < 2; ++s)
            if (s ? qv1[k] : qv0[k]) {
                const int li = tile_slot(qx[k] + s, qy[k], (rx0 + ry0 + qx[k] + s + qy[k]) & 1, pw);
                sFA[li] = lf[k][s];
                sB[li] = lb[k][s];
            }
    lds_sync();

    if constexpr (EN) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kTilePairsPerThread; ++k)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int x = qx[k] + s, y = qy[k], gx = rx0 + x, gy = ry0 + y;
                if (!(s ? qv1[k] : qv0[k]) || gx < R.cx0 || gx >= R.cx1 || gy < R.cy0 || gy >= R.cy1)
                    continue;
                const float4 f = lf[k][s], g = lb[k][s];
                const float a = f.w, b = 1.0f - a;
                const float fv[3] = {f.x, f.y, f.z}, bv[3] = {g.x, g.y, g.z};
                float e = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float res = fmaf(a, fv[c], fmaf(b, bv[c], -in.iv[k][s][c]));
                    e = fmaf(res, res, e);
                }
#pragma unroll
                for (int dir = 0; dir < 2; ++dir) {
                    if (dir == 0 ? gx + 1 >= w : gy + 1 >= h) continue;
                    const int nx = x + (dir == 0), ny = y + (dir == 1);
                    const int j = tile_slot(nx, ny, (rx0 + ry0 + nx + ny) & 1, pw);
                    const float4 fj = sFA[j], gj = sB[j];
                    const float fjv[3] = {fj.x, fj.y, fj.z}, bjv[3] = {gj.x, gj.y, gj.z};
                    float d = 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float df = fv[c] - fjv[c], db = bv[c] - bjv[c];
                        d = fmaf(df, df, fmaf(db, db, d));
                    }
                    e = fmaf(fmaf(omega, fabsf(a - fj.w), eps), d, e);
                }
                acc += static_cast<double>(e);
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((tid & 63) == 0) ered[tid >> 6] = acc;
        lds_sync();   // also: every neighbour read above is done before the sweeps write
        if (tid == 0) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < kTileThreads / 64; ++q) sum += ered[q];
            double *o = epart + 5 * static_cast<size_t>(unit);
            o[0] = sum;
            o[1] = o[2] = o[3] = o[4] = 0.0;
        }
    }

    // Weights of the pixel updated in half-sweep c of each pair (colour-ordered, as in the
    // coarse kernel): slot (rx0 + ry0 + y + c) & 1 of the pair.
    int cpix[kTilePairsPerThread][2], cnb[kTilePairsPerThread][2][4];
    bool cok[kTilePairsPerThread][2];
    float cw[kTilePairsPerThread][2][4], cka[kTilePairsPerThread][2], ckb[kTilePairsPerThread][2];
    float ca[kTilePairsPerThread][2], ci[kTilePairsPerThread][2][3];
#pragma unroll
    for (int k = 0; k < kTilePairsPerThread; ++k) {
        int tnb[2][4];
        float tw[2][4], tka[2], tkb[2], ta[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int x = min(qx[k] + s, rw - 1), y = min(qy[k], rh - 1);
            const int g = (rx0 + ry0 + x + y) & 1;   // this pixel's colour; neighbours have 1 - g
            const int i = tile_slot(x, y, g, pw);
            tnb[s][0] = x > 0 ? tile_slot(x - 1, y, g ^ 1, pw) : i;
            tnb[s][1] = x < rw - 1 ? tile_slot(x + 1, y, g ^ 1, pw) : i;
            tnb[s][2] = y > 0 ? tile_slot(x, y - 1, g ^ 1, pw) : i;
            tnb[s][3] = y < rh - 1 ? tile_slot(x, y + 1, g ^ 1, pw) : i;
            const float a = sFA[i].w;
            float sj[4], S = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sj[j] = weight(a, sFA[tnb[s][j]].w, omega, eps);
                S += sj[j];
            }
            const float iS = rcp(S), b = 1.0f - a;
            const float kk = rcp(S + fmaf(a, a, b * b));
#pragma unroll
            for (int j = 0; j < 4; ++j) tw[s][j] = sj[j] * iS;
            tka[s] = a * kk;
            tkb[s] = b * kk;
            ta[s] = a;
        }
        const bool flip = (rx0 + ry0 + qy[k]) & 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bool hi = flip ? (c == 0) : (c == 1);
            cpix[k][c] = tile_slot(qx[k] + (hi ? 1 : 0), qy[k], c, pw);
            cok[k][c] = hi ? qv1[k] : qv0[k];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cnb[k][c][j] = hi ? tnb[1][j] : tnb[0][j];
                cw[k][c][j] = hi ? tw[1][j] : tw[0][j];
            }
            cka[k][c] = hi ? tka[1] : tka[0];
            ckb[k][c] = hi ? tkb[1] : tkb[0];
            ca[k][c] = hi ? ta[1] : ta[0];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) ci[k][c][ch] = hi ? in.iv[k][1][ch] : in.iv[k][0][ch];
        }
    }

    // The update of the colour-c pixel of each owned pair from the neighbours in LDS.
    // Unconditional reads and arithmetic (indices are clamped into the region), guarded stores:
    // the reads of all owned pairs are in flight together.
    auto solve = [&](int c, float (&fo)[kTilePairsPerThread][3], float (&bo)[kTilePairsPerThread][3]) {
#pragma unroll
        for (int k = 0; k < kTilePairsPerThread; ++k) {
            float fb[3] = {0.f, 0.f, 0.f}, bb[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float wj = cw[k][c][j];
                const float4 f = sFA[cnb[k][c][j]];
                const float4 g = sB[cnb[k][c][j]];
                fb[0] = fmaf(wj, f.x, fb[0]);
                fb[1] = fmaf(wj, f.y, fb[1]);
                fb[2] = fmaf(wj, f.z, fb[2]);
                bb[0] = fmaf(wj, g.x, bb[0]);
                bb[1] = fmaf(wj, g.y, bb[1]);
                bb[2] = fmaf(wj, g.z, bb[2]);
            }
            const float a = ca[k][c], b = 1.0f - a;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float r = ci[k][c][ch] - a * fb[ch] - b * bb[ch];
                fo[k][ch] = clamp01(fmaf(cka[k][c], r, fb[ch]));
                bo[k][ch] = clamp01(fmaf(ckb[k][c], r, bb[ch]));
            }
        }
    };
    auto put = [&](int c, const float (&fo)[kTilePairsPerThread][3],
                   const float (&bo)[kTilePairsPerThread][3]) {
#pragma unroll
        for (int k = 0; k < kTilePairsPerThread; ++k)
            if (cok[k][c]) {
                sFA[cpix[k][c]] = make_float4(fo[k][0], fo[k][1], fo[k][2], ca[k][c]);
                sB[cpix[k][c]] = make_float4(bo[k][0], bo[k][1], bo[k][2], 0.0f);
            }
    };
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        if constexpr (JAC) {
            // Jacobi: both colours from the state before the sweep, written after every read
            // of the sweep (each sweep invalidates one ring of the region; two are needed).
            float fo0[kTilePairsPerThread][3], bo0[kTilePairsPerThread][3];
            float fo1[kTilePairsPerThread][3], bo1[kTilePairsPerThread][3];
            solve(0, fo0, bo0);
            solve(1, fo1, bo1);
            lds_sync();
            put(0, fo0, bo0);
            put(1, fo1, bo1);
            lds_sync();
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float fo[kTilePairsPerThread][3], bo[kTilePairsPerThread][3];
                solve(c, fo, bo);
                put(c, fo, bo);
                lds_sync();
            }
        }
    }

    if (!Fo) return;
    // Store the core.
    const size_t planeO = static_cast<size_t>(w) * h;
    const int cw_ = R.cx1 - R.cx0, ch_ = R.cy1 - R.cy0;
    const float rcw_ = rcp(static_cast<float>(cw_));
    for (int p = tid; p < cw_ * ch_; p += kTileThreads) {
        const int yy = fdiv(p, cw_, rcw_), xx = p - yy * cw_;
        const int gx = R.cx0 + xx, gy = R.cy0 + yy;
        const int li = tile_slot(gx - rx0, gy - ry0, (gx + gy) & 1, pw);
        const float4 f = sFA[li], g = sB[li];
        const size_t o = static_cast<size_t>(gy) * w + gx;
        stf(Fo + o, f.x);
        stf(Fo + planeO + o, f.y);
        stf(Fo + 2 * planeO + o, f.z);
        stf(Bo + o, g.x);
        stf(Bo + planeO + o, g.y);
        stf(Bo + 2 * planeO + o, g.z);
    }
}

// One fine level, output tile `tile`: the level's F and B come from the stored previous level.
template <typename T, bool EN = false, bool JAC = false>
__device__ __forceinline__ void tile_body(const TileArgs &args, int tile, TileLds &lds,
                                          double *epart = nullptr, double *ered = nullptr) {
    const int w = args.w, h = args.h;
    const int tx = tile % args.tiles_x, ty = tile / args.tiles_x;
    const int cx0 = tx * kTileCore, cy0 = ty * kTileCore;
    const TileRegion R = tile_region(cx0, min(w, cx0 + kTileCore), cy0, min(h, cy0 + kTileCore), w, h);
    TilePrev pv{};
    pv.Fp = args.Fp;
    pv.Bp = args.Bp;
    pv.wp = args.wp;
    pv.hp = args.hp;
    TileInput in;
    tile_fetch<T>(static_cast<const T *>(args.I), static_cast<const T *>(args.A), args.W, args.H,
                  w, h, R, in);
    tile_level<T, false, EN, JAC>(in, w, h, pv, R, lds.FA, lds.B, args.omega, args.eps,
                                  static_cast<T *>(args.Fo), static_cast<T *>(args.Bo), epart, tile,
                                  ered);
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void tile_kernel(TileArgs args) {
    __shared__ TileLds lds;
    tile_body<T>(args, blockIdx.x, lds);
}

// The convergence form's passes (float32 state): a tile pass that also reduces the energy of
// the state it starts from, one partial per tile; JAC: its two sweeps in the Jacobi order.  A
// non-null `skip` holding a non-zero value (the level has stopped) makes the launch a no-op.
template <bool JAC>
__global__ __launch_bounds__(kTileThreads) void tile_energy_kernel(TileArgs args, double *epart,
                                                                  const int *skip) {
    if (skip && *skip) return;
    __shared__ TileLds lds;
    __shared__ double ered[kTileThreads / 64];
    tile_body<float, true, JAC>(args, blockIdx.x, lds, epart, ered);
}

// ------------------------------------------------------------------------------------------
// Pyramid kernel: a run of consecutive tile levels in one launch.
// ------------------------------------------------------------------------------------------
//
// Workgroup t owns output tile t of the run's last level and computes, from the run's first
// level up, exactly the region of each level its tile depends on: the last level's region is
// the tile plus its ring; a lower level's core is the set of rows and columns the nearest map of
// the level above reads over that region (an interval: the map is monotone), and its region
// that core plus its own ring.  Each level's region stays in LDS for the next one; only the
// first level reads a stored previous level and only the last stores its core.  Neighbouring
// workgroups recompute overlapping lower-level regions; in exchange the run is one launch, not
// one per level, and its intermediate levels never go through memory.  Every level uses the
// tile kernel's arithmetic, so the stored values are bit-identical to a per-level run.

// Regions of the run for output tile `tile` (levels 0..nl-1 of the run, last = output level).
// The host (pyramid_fits) evaluates the same function to check that every region fits LDS.
__host__ __device__ inline void pyramid_regions(const PyramidArgs &a, int tile, TileRegion *R) {
    // Level sizes first, at fixed indices (on the device: every argument load in flight at once).
    const int L = a.nl;
    int lw[kPyrMaxLevels], lh[kPyrMaxLevels];
#pragma unroll
    for (int l = 0; l < kPyrMaxLevels; ++l) {
        lw[l] = a.lv[l].w;
        lh[l] = a.lv[l].h;
    }
    int cx0 = 0, cx1 = 0, cy0 = 0, cy1 = 0;
#pragma unroll
    for (int l = kPyrMaxLevels - 1; l >= 0; --l) {
        if (l >= L) continue;
        const int w = lw[l], h = lh[l];
        if (l == L - 1) {   // the output tile
            const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
            cx0 = tx * kTileCore;
            cy0 = ty * kTileCore;
            cx1 = cx0 + kTileCore < w ? cx0 + kTileCore : w;
            cy1 = cy0 + kTileCore < h ? cy0 + kTileCore : h;
        }
        TileRegion r;
        r.cx0 = cx0;
        r.cx1 = cx1;
        r.cy0 = cy0;
        r.cy1 = cy1;
        r.rx0 = cx0 - kTileHalo > 0 ? cx0 - kTileHalo : 0;
        r.ry0 = cy0 - kTileHalo > 0 ? cy0 - kTileHalo : 0;
        r.rw = (cx1 + kTileHalo < w ? cx1 + kTileHalo : w) - r.rx0;
        r.rh = (cy1 + kTileHalo < h ? cy1 + kTileHalo : h) - r.ry0;
        R[l] = r;
        if (l > 0) {   // the part of the level below that the nearest map reads over r
            const int wp = lw[l - 1], hp = lh[l - 1];
            cx0 = r.rx0 * wp / w;
            cx1 = (r.rx0 + r.rw - 1) * wp / w + 1;
            cy0 = r.ry0 * hp / h;
            cy1 = (r.ry0 + r.rh - 1) * hp / h + 1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void pyramid_kernel(PyramidArgs args) {
    __shared__ TileLds buf[2];
    __shared__ TileRegion sR[kPyrMaxLevels];
    if (threadIdx.x == 0) pyramid_regions(args, blockIdx.x, sR);
    lds_sync();
    const int L = args.nl;
    // Each level's inputs are fetched one level ahead: their gathers run during the sweeps of
    // the level before (the workgroup barriers wait for LDS only).
    TileInput cur, nxt;
    tile_fetch<T>(static_cast<const T *>(args.lv[0].I), static_cast<const T *>(args.lv[0].A),
                  args.lv[0].W, args.lv[0].H, args.lv[0].w, args.lv[0].h, sR[0], cur);
    for (int l = 0; l < L; ++l) {
        const PyramidLevel &d = args.lv[l];
        const TileRegion R = sR[l];
        if (l + 1 < L) {
            const PyramidLevel &e = args.lv[l + 1];
            tile_fetch<T>(static_cast<const T *>(e.I), static_cast<const T *>(e.A), e.W, e.H, e.w,
                          e.h, sR[l + 1], nxt);
        }
        T *Fo = l == L - 1 ? static_cast<T *>(args.Fo) : nullptr;
        T *Bo = l == L - 1 ? static_cast<T *>(args.Bo) : nullptr;
        TilePrev pv{};
        if (l == 0) {
            pv.Fp = args.Fp;
            pv.Bp = args.Bp;
            pv.wp = args.wp;
            pv.hp = args.hp;
            tile_level<T, false>(cur, d.w, d.h, pv, R, buf[0].FA, buf[0].B, args.omega, args.eps,
                                 Fo, Bo);
        } else {
            const TileRegion P = sR[l - 1];
            pv.sFA = buf[(l - 1) & 1].FA;
            pv.sB = buf[(l - 1) & 1].B;
            pv.rx0 = P.rx0;
            pv.ry0 = P.ry0;
            pv.pw = (P.rw + 1) >> 1;
            pv.wp = args.lv[l - 1].w;
            pv.hp = args.lv[l - 1].h;
            tile_level<T, true>(cur, d.w, d.h, pv, R, buf[l & 1].FA, buf[l & 1].B, args.omega,
                                args.eps, Fo, Bo);
        }
        cur = nxt;
    }
}


// ------------------------------------------------------------------------------------------
// Naive path: upsample, then one launch per half-sweep.
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ void upsample_kernel(const T *Fp, const T *Bp, int wp, int hp, T *Fo, T *Bo, int w,
                                int h) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= w * h) return;
    const int y = p / w, x = p - y * w;
    const size_t n = static_cast<size_t>(w) * h, np = static_cast<size_t>(wp) * hp;
    const int q = (y * hp / h) * wp + x * wp / w;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        stf(Fo + c * n + p, Fp ? ldf(Fp + c * np + q) : 0.0f);
        stf(Bo + c * n + p, Bp ? ldf(Bp + c * np + q) : 0.0f);
    }
}

template <typename T>
__global__ void halfsweep_kernel(const T *I, const T *A, int W, int H, T *F, T *B, int w, int h,
                                 int colour, float omega, float eps) {
    const int pw = (w + 1) >> 1;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= pw * h) return;
    const int y = q / pw;
    const int x = 2 * (q - y * pw) + ((y + colour) & 1);
    if (x >= w) return;
    const size_t n = static_cast<size_t>(w) * h, planeI = static_cast<size_t>(W) * H;
    const int rowI = y * H / h;
    auto alpha_at = [&](int xx, int yy) {
        return ldf(A + static_cast<size_t>(yy * H / h) * W + xx * W / w);
    };
    const float a = alpha_at(x, y);
    const int xs[4] = {x > 0 ? x - 1 : 0, x < w - 1 ? x + 1 : w - 1, x, x};
    const int ys[4] = {y, y, y > 0 ? y - 1 : 0, y < h - 1 ? y + 1 : h - 1};
    float s[4], S = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        s[j] = weight(a, alpha_at(xs[j], ys[j]), omega, eps);
        S += s[j];
    }
    const float iS = 1.0f / S, b = 1.0f - a;
    const float k = 1.0f / (S + fmaf(a, a, b * b));
    const size_t i = static_cast<size_t>(y) * w + x;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float P = 0.0f, Q = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t nj = c * n + static_cast<size_t>(ys[j]) * w + xs[j];
            P = fmaf(s[j], ldf(F + nj), P);
            Q = fmaf(s[j], ldf(B + nj), Q);
        }
        const float fb = P * iS, bb = Q * iS;
        const float r = ldf(I + c * planeI + static_cast<size_t>(rowI) * W + x * W / w) - a * fb - b * bb;
        stf(F + c * n + i, clamp01(fmaf(a * k, r, fb)));
        stf(B + c * n + i, clamp01(fmaf(b * k, r, bb)));
    }
}

// ------------------------------------------------------------------------------------------
// Fused fine-level kernel: streaming red-black sweeps on a register window.
// ------------------------------------------------------------------------------------------

constexpr int kNHS = 4;                 // half-sweeps per level (two sweeps)
constexpr int kPD = 2;                  // rows loaded ahead of the row being consumed
constexpr int kWin = kNHS + 2 + kPD;    // rows held per wave: t-5 .. t+kPD
constexpr int kHalo = kNHS;             // invalid ring after kNHS half-sweeps
constexpr int kStripCols = 128;         // two columns per lane
constexpr int kFirstCore = kStripCols - kHalo;          // strip 0 keeps columns [0, 124)
constexpr int kMidCore = kStripCols - 2 * kHalo;        // interior strips keep 120 columns
constexpr int kWavesPerBlock = 4;
constexpr int kXcds = 8;                // accelerator dies, one L2 each
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer resource, gfx9 family


// Number of column strips for a level of width w (see the geometry in fine_strip).
__host__ __device__ inline int fine_strips_x(int w) {
    if (w <= kStripCols) return 1;
    const int rest = w - (kFirstCore + kFirstCore);
    return 2 + (rest > 0 ? (rest + kMidCore - 1) / kMidCore : 0);
}

// Raw buffer resource over `bytes` bytes (< 4 GiB, checked by the planner).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tensor_rsrc(const void *base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0,
                                             static_cast<int>(static_cast<uint32_t>(bytes)),
                                             kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ uint32_t bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<int>(voff), static_cast<int>(soff), 0);
}

// Float-typed raw buffer loads (the LLVM intrinsics directly): the register window then only
// ever holds floats, which keeps it promotable to registers.
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ float raw_load_f32(__amdgpu_buffer_rsrc_t r, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.load.f32");
__device__ f32x2 raw_load_v2f32(__amdgpu_buffer_rsrc_t r, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.load.v2f32");

__device__ __forceinline__ float loadf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return raw_load_f32(r, static_cast<int>(voff), static_cast<int>(soff), 0);
}
__device__ __forceinline__ f32x2 loadf2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return raw_load_v2f32(r, static_cast<int>(voff), static_cast<int>(soff), 0);
}

template <typename T>
__device__ __forceinline__ float bits_to_float(uint32_t v) {
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(v);
    } else {
        const unsigned short hb = static_cast<unsigned short>(v);
        return static_cast<float>(__builtin_bit_cast(_Float16, hb));
    }
}

template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, static_cast<int>(voff),
                                              static_cast<int>(soff), 0);
    } else {
        const _Float16 hv = static_cast<_Float16>(v);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hv), r,
                                              static_cast<int>(voff), static_cast<int>(soff), 0);
    }
}

// Lane i receives v from lane i-1; lane 0 receives 0 (DPP wave_shr:1 with bound control), a
// form the compiler can fold into the consuming FMA.  Only used where lane 0 is halo.
__device__ __forceinline__ float from_left_z(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Lane i receives v from lane i+1; lane 63 receives 0.
__device__ __forceinline__ float from_right_z(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// Per-wave constants of a strip.  Each tensor (I, alpha, previous F and B, F, B) is one buffer
// resource (the previous level's F and B are one workspace buffer, B right after F); a load takes the row's byte offset plus the plane's byte offset as the scalar
// offset and the lane's column as the (loop-invariant) vector offset, so there is no per-row
// vector address arithmetic.  The planner sends a level here only when every tensor is below
// 4 GiB, the reach of a buffer resource.
struct FineGeo {
    __amdgpu_buffer_rsrc_t I, A, P, Fo, Bo;   // P: previous F (planes 0-2) then B (3-5)
    uint32_t pI, pP, pO;           // plane sizes in bytes (input, previous level, output)
    int W, H, wp, hp, w, h;
    uint32_t sia, sib, spa, spb;   // byte offsets of this lane's source columns
    uint32_t oxa, oxb;             // byte offsets of this lane's output columns
    bool store_a, store_b;         // columns inside this strip's core
    bool left_a;                   // column a == 0 (left image border inside the wave)
    bool right_a, right_b;         // column == w - 1 (right image border inside the wave)
    int y0, y1, t0, tlast;
    float omega, eps;
};

// Register window: row slot = (row - t0) mod kWin, column of the lane's pair.  Rows are loaded
// kPD steps ahead straight into their slot as raw bits (float32: final values; binary16:
// converted when the row is consumed).
struct FineWin {
    uint32_t ra[kWin][2], ri[kWin][2][3], rf[kWin][2][3], rb[kWin][2][3];
    float al[kWin][2];
    float iv[kWin][2][3];
    float fv[kWin][2][3];
    float bv[kWin][2][3];
    float wl[kWin][2], wr[kWin][2], wu[kWin][2], wd[kWin][2], ka[kWin][2], kb[kWin][2];
    double energy;   // the energy kernels only: this lane's share of the input state's energy
};

// floor(tc * num / den) for a row index tc that advances one at a time (uniform, no division).
struct RowMap {
    int q, r, qd, rd, den;
    __device__ void init(int tc, int num, int d) {
        den = d;
        qd = num / d;
        rd = num - qd * d;
        const long long v = static_cast<long long>(tc) * num;
        q = static_cast<int>(v / d);
        r = static_cast<int>(v - static_cast<long long>(q) * d);
    }
    __device__ __forceinline__ void advance() {
        q += qd;
        r += rd;
        if (r >= den) {
            r -= den;
            q += 1;
        }
    }
};

// Access paths of a streaming strip (template parameter PAIR):
//   kPairNone  every pixel loads and stores on its own (strips at an image border, odd widths);
//   kPairIn    the input map is the identity in x and the strip starts on an even column: a
//              lane's two columns are adjacent in I and alpha (one load per plane) and in F and
//              B (one store per plane); the previous level is read per pixel;
//   kPairFull  as kPairIn, and the previous level is exactly half as wide: both columns read
//              the same previous-level column (one load per plane);
//   kPairSame  as kPairIn, and the previous state has the level's own size (the passes of the
//              convergence form after the first): a lane's two columns are adjacent there too
//              (one load per plane).
constexpr int kPairNone = 0, kPairIn = 1, kPairFull = 2, kPairSame = 3;

// Gather one row into slot R: I and alpha from input row qi (nearest), F and B from
// previous-level row qp.  float32 lands in the float window directly; binary16 lands as raw
// bits and is converted when the row is consumed.
template <int R, int PAIR, typename T>
__device__ __forceinline__ void fine_load_row(FineWin &v, const FineGeo &g, int qi, int qp) {
    const uint32_t si = static_cast<uint32_t>(qi) * static_cast<uint32_t>(g.W) * sizeof(T);
    const uint32_t sp = static_cast<uint32_t>(qp) * static_cast<uint32_t>(g.wp) * sizeof(T);
    if constexpr (sizeof(T) == 4) {
        if constexpr (PAIR >= kPairIn) {
            const f32x2 av = loadf2(g.A, g.sia, si);
            v.al[R][0] = av.x;
            v.al[R][1] = av.y;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const f32x2 iv = loadf2(g.I, g.sia, si + c * g.pI);
                v.iv[R][0][c] = iv.x;
                v.iv[R][1][c] = iv.y;
            }
        } else {
            v.al[R][0] = loadf(g.A, g.sia, si);
            v.al[R][1] = loadf(g.A, g.sib, si);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t ci = si + c * g.pI;
                v.iv[R][0][c] = loadf(g.I, g.sia, ci);
                v.iv[R][1][c] = loadf(g.I, g.sib, ci);
            }
        }
        if constexpr (PAIR == kPairFull) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                v.fv[R][0][c] = v.fv[R][1][c] = loadf(g.P, g.spa, cp);
                v.bv[R][0][c] = v.bv[R][1][c] = loadf(g.P, g.spa, cp + 3 * g.pP);
            }
        } else if constexpr (PAIR == kPairSame) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                const f32x2 fv = loadf2(g.P, g.spa, cp), bv = loadf2(g.P, g.spa, cp + 3 * g.pP);
                v.fv[R][0][c] = fv.x;
                v.fv[R][1][c] = fv.y;
                v.bv[R][0][c] = bv.x;
                v.bv[R][1][c] = bv.y;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                v.fv[R][0][c] = loadf(g.P, g.spa, cp);
                v.fv[R][1][c] = loadf(g.P, g.spb, cp);
                v.bv[R][0][c] = loadf(g.P, g.spa, cp + 3 * g.pP);
                v.bv[R][1][c] = loadf(g.P, g.spb, cp + 3 * g.pP);
            }
        }
    } else {
        if constexpr (PAIR >= kPairIn) {
            const uint32_t av = bload<float>(g.A, g.sia, si);
            v.ra[R][0] = av;
            v.ra[R][1] = av >> 16;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t iv = bload<float>(g.I, g.sia, si + c * g.pI);
                v.ri[R][0][c] = iv;
                v.ri[R][1][c] = iv >> 16;
            }
        } else {
            v.ra[R][0] = bload<T>(g.A, g.sia, si);
            v.ra[R][1] = bload<T>(g.A, g.sib, si);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t ci = si + c * g.pI;
                v.ri[R][0][c] = bload<T>(g.I, g.sia, ci);
                v.ri[R][1][c] = bload<T>(g.I, g.sib, ci);
            }
        }
        if constexpr (PAIR == kPairFull) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                v.rf[R][0][c] = v.rf[R][1][c] = bload<T>(g.P, g.spa, cp);
                v.rb[R][0][c] = v.rb[R][1][c] = bload<T>(g.P, g.spa, cp + 3 * g.pP);
            }
        } else if constexpr (PAIR == kPairSame) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                const uint32_t fv = bload<float>(g.P, g.spa, cp), bv = bload<float>(g.P, g.spa, cp + 3 * g.pP);
                v.rf[R][0][c] = fv;
                v.rf[R][1][c] = fv >> 16;
                v.rb[R][0][c] = bv;
                v.rb[R][1][c] = bv >> 16;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t cp = sp + c * g.pP;
                v.rf[R][0][c] = bload<T>(g.P, g.spa, cp);
                v.rf[R][1][c] = bload<T>(g.P, g.spb, cp);
                v.rb[R][0][c] = bload<T>(g.P, g.spa, cp + 3 * g.pP);
                v.rb[R][1][c] = bload<T>(g.P, g.spb, cp + 3 * g.pP);
            }
        }
    }
}

template <int R, typename T>
__device__ __forceinline__ void fine_consume(FineWin &v) {
    if constexpr (sizeof(T) == 4) return;   // already final
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        v.al[R][s] = bits_to_float<T>(v.ra[R][s]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v.iv[R][s][c] = bits_to_float<T>(v.ri[R][s][c]);
            v.fv[R][s][c] = bits_to_float<T>(v.rf[R][s][c]);
            v.bv[R][s][c] = bits_to_float<T>(v.rb[R][s][c]);
        }
    }
}

// Horizontal neighbours of the pair's two pixels from a per-lane value pair (a, b):
// left of a is lane-1's b, right of b is lane+1's a.  EDGE strips contain an image border: there
// the clamp makes the border pixel its own neighbour; elsewhere the wave-edge lanes are halo.
template <bool EDGE>
__device__ __forceinline__ float left_of_a(const FineGeo &g, float a, float b) {
    const float l = from_left_z(b);
    return EDGE && g.left_a ? a : l;
}
template <bool EDGE>
__device__ __forceinline__ float right_of_b(const FineGeo &g, float a, float b) {
    const float r = from_right_z(a);
    return EDGE && g.right_b ? b : r;
}
template <bool EDGE>
__device__ __forceinline__ float right_of_a(const FineGeo &g, float a, float b) {
    return EDGE && g.right_a ? a : b;
}

// Weights of row r (slot R) from its own and its neighbours' alpha (rows in slots U and D).
// Rows -1 and h are phantom rows outside the image: the neighbour clamp of Algorithm 1 makes a
// border pixel its own neighbour, and the phantom row holds exactly that value, because its
// "update" copies the adjacent image row (weights 1 toward it, 0 elsewhere, no data term).
// Rows beyond the phantom rows are loaded from the clamped border row and never feed a stored
// result.
template <int R, int U, int D, bool EDGE, bool BORDER>
__device__ __forceinline__ void fine_constants(FineWin &v, const FineGeo &g, int r) {
    const float omega = g.omega, eps = g.eps;
    const float a0 = v.al[R][0], a1 = v.al[R][1];
    const float l0 = left_of_a<EDGE>(g, a0, a1);
    const float r0 = right_of_a<EDGE>(g, a0, a1);
    const float r1 = right_of_b<EDGE>(g, a0, a1);
    const float mid = weight(a0, r0, omega, eps);      // edge between the lane's two columns
    const float sl[2] = {weight(a0, l0, omega, eps), EDGE ? weight(a1, a0, omega, eps) : mid};
    const float sr[2] = {mid, weight(a1, r1, omega, eps)};
    const bool copy_down = BORDER && r == -1;
    const bool copy_up = BORDER && r == g.h;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float a = v.al[R][s];
        const float su = weight(a, v.al[U][s], omega, eps);
        const float sd = weight(a, v.al[D][s], omega, eps);
        const float S = (sl[s] + sr[s]) + (su + sd);
        const float iS = rcp(S);
        const float b = 1.0f - a;
        const float k = rcp(S + fmaf(a, a, b * b));
        float cl = sl[s] * iS, cr = sr[s] * iS, cu = su * iS, cd = sd * iS;
        float ca = a * k, cb = b * k;
        if (BORDER && (copy_down || copy_up)) {
            cl = cr = ca = cb = 0.0f;
            cu = copy_up ? 1.0f : 0.0f;
            cd = copy_down ? 1.0f : 0.0f;
        }
        v.wl[R][s] = cl;
        v.wr[R][s] = cr;
        v.wu[R][s] = cu;
        v.wd[R][s] = cd;
        v.ka[R][s] = ca;
        v.kb[R][s] = cb;
    }
}

// Half-sweep on the row in slot R: update column S of every lane.
template <int R, int U, int D, int S, bool EDGE>
__device__ __forceinline__ void fine_update(FineWin &v, const FineGeo &g) {
    const float a = v.al[R][S], b = 1.0f - a;
    const float cl = v.wl[R][S], cr = v.wr[R][S], cu = v.wu[R][S], cd = v.wd[R][S];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float fL, fR, bL, bR;
        if (S == 0) {
            fL = left_of_a<EDGE>(g, v.fv[R][0][c], v.fv[R][1][c]);
            bL = left_of_a<EDGE>(g, v.bv[R][0][c], v.bv[R][1][c]);
            fR = right_of_a<EDGE>(g, v.fv[R][0][c], v.fv[R][1][c]);
            bR = right_of_a<EDGE>(g, v.bv[R][0][c], v.bv[R][1][c]);
        } else {
            fL = v.fv[R][0][c];
            bL = v.bv[R][0][c];
            fR = right_of_b<EDGE>(g, v.fv[R][0][c], v.fv[R][1][c]);
            bR = right_of_b<EDGE>(g, v.bv[R][0][c], v.bv[R][1][c]);
        }
        // The lane-shifted neighbour (left for column a, right for column b) enters through the
        // first product, a plain multiply into which the DPP move folds.
        float fb, bb;
        if (S == 0) {
            fb = fmaf(cd, v.fv[D][S][c], fmaf(cu, v.fv[U][S][c], fmaf(cr, fR, cl * fL)));
            bb = fmaf(cd, v.bv[D][S][c], fmaf(cu, v.bv[U][S][c], fmaf(cr, bR, cl * bL)));
        } else {
            fb = fmaf(cd, v.fv[D][S][c], fmaf(cu, v.fv[U][S][c], fmaf(cl, fL, cr * fR)));
            bb = fmaf(cd, v.bv[D][S][c], fmaf(cu, v.bv[U][S][c], fmaf(cl, bL, cr * bR)));
        }
        const float r = v.iv[R][S][c] - a * fb - b * bb;
        v.fv[R][S][c] = clamp01(fmaf(v.ka[R][S], r, fb));
        v.bv[R][S][c] = clamp01(fmaf(v.kb[R][S], r, bb));
    }
}

// The energy of the state a pass starts from, accumulated while it streams (the energy kernels):
// at step t, after row t is taken and before row t - 1's first half-sweep, rows t - 1 and t still
// hold that state.  Row r = t - 1 (slot R, row r + 1 in slot D) adds, for each core pixel of the
// lane, its data term and its right and lower edges (so every edge of the level once), each
// pixel's terms summed in float32 and added to the lane's float64 total.
template <int R, int D, bool EDGE>
__device__ __forceinline__ void fine_energy(FineWin &v, const FineGeo &g, int r) {
    if (r < g.y0 || r >= g.y1) return;   // core rows (wave-uniform)
    const float omega = g.omega, eps = g.eps;
    const bool down = r + 1 < g.h;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float a = v.al[R][s], b = 1.0f - a;
        float e = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float res = fmaf(a, v.fv[R][s][c], fmaf(b, v.bv[R][s][c], -v.iv[R][s][c]));
            e = fmaf(res, res, e);
        }
        // right neighbour: column b of the lane, or column a of the next lane
        const float ar = s == 0 ? v.al[R][1] : from_right_z(v.al[R][0]);
        float dr = 0.0f, dd = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float fr = s == 0 ? v.fv[R][1][c] : from_right_z(v.fv[R][0][c]);
            const float br = s == 0 ? v.bv[R][1][c] : from_right_z(v.bv[R][0][c]);
            const float df = v.fv[R][s][c] - fr, db = v.bv[R][s][c] - br;
            dr = fmaf(df, df, fmaf(db, db, dr));
            const float dfd = v.fv[R][s][c] - v.fv[D][s][c], dbd = v.bv[R][s][c] - v.bv[D][s][c];
            dd = fmaf(dfd, dfd, fmaf(dbd, dbd, dd));
        }
        const bool right = s == 0 ? !g.right_a : !g.right_b;
        if (right) e = fmaf(fmaf(omega, fabsf(a - ar), eps), dr, e);
        if (down) e = fmaf(fmaf(omega, fabsf(a - v.al[D][s]), eps), dd, e);
        if (s == 0 ? g.store_a : g.store_b) v.energy += static_cast<double>(e);
    }
}

template <typename T>
__device__ __forceinline__ void bstore_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                            float v0, float v1) {
    // non-temporal: the finest level's F and B are not read again by this pass
    if constexpr (sizeof(T) == 4) {
        // The empty asm pins the two values as separate registers: otherwise the compiler reads
        // them from the window as one vector, which keeps the window out of registers.
        asm volatile("" : "+v"(v0), "+v"(v1));
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 d = {__float_as_uint(v0), __float_as_uint(v1)};
        __builtin_amdgcn_raw_buffer_store_b64(d, r, static_cast<int>(voff), static_cast<int>(soff), 2);
    } else {
        // One vector conversion: gfx950 converts and packs the pair in a single instruction,
        // rounding each value to nearest even as a scalar conversion does.
        typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
        asm volatile("" : "+v"(v0), "+v"(v1));   // as above: keeps the window in registers
        const f32x2 fv = {v0, v1};
        const f16x2 hv = __builtin_convertvector(fv, f16x2);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, hv), r,
                                              static_cast<int>(voff), static_cast<int>(soff), 2);
    }
}

template <int R, int PAIR, typename T>
__device__ __forceinline__ void fine_store_row(const FineWin &v, const FineGeo &g, int r) {
    const uint32_t so = static_cast<uint32_t>(r) * static_cast<uint32_t>(g.w) * sizeof(T);
    if constexpr (PAIR >= kPairIn) {
        if (g.store_a) {   // == store_b: core boundaries are even in a paired strip
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bstore_pair<T>(g.Fo, g.oxa, so + c * g.pO, v.fv[R][0][c], v.fv[R][1][c]);
                bstore_pair<T>(g.Bo, g.oxa, so + c * g.pO, v.bv[R][0][c], v.bv[R][1][c]);
            }
        }
        return;
    }
    if (g.store_a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            bstore<T>(g.Fo, g.oxa, so + c * g.pO, v.fv[R][0][c]);
            bstore<T>(g.Bo, g.oxa, so + c * g.pO, v.bv[R][0][c]);
        }
    }
    if (g.store_b) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            bstore<T>(g.Fo, g.oxb, so + c * g.pO, v.fv[R][1][c]);
            bstore<T>(g.Bo, g.oxb, so + c * g.pO, v.bv[R][1][c]);
        }
    }
}

// One pipeline step at row t (TT = (t - t0) mod kWin): load row t + kPD (clamped into the image)
// into its slot, take row t, compute the weights of row t-1, run half-sweep k on row t-1-k for
// k = 0..3, and store row t-4, which has now seen both sweeps.  ST says what the caller knows of
// row t-4: kStNone, outside the core (no store); kStCore, inside (an unconditional store);
// kStCheck, either (tested at run time).  A branch around a memory access costs more than its
// test: the wait counters must assume the worst where the paths join, which makes a later step
// wait for the prefetch of its own rows.
constexpr int kStCheck = 0, kStNone = 1, kStCore = 2;
template <int TT, bool EDGE, bool BORDER, int PAIR, typename T, int ST, bool EN>
__device__ __forceinline__ void fine_step(FineWin &v, const FineGeo &g, RowMap &mi, RowMap &mp,
                                          int t) {
    constexpr int S = (TT + 1) & 1;       // column of the pair updated in this step
    {
        const int tl = t + kPD;
        if (tl >= 1 && tl <= g.h - 1) {
            mi.advance();
            mp.advance();
        }
        fine_load_row<(TT + kPD) % kWin, PAIR, T>(v, g, mi.q, mp.q);
    }
    fine_consume<TT % kWin, T>(v);
    if constexpr (EN) fine_energy<(TT + kWin - 1) % kWin, TT % kWin, EDGE>(v, g, t - 1);
    fine_constants<(TT + kWin - 1) % kWin, (TT + kWin - 2) % kWin, TT % kWin, EDGE, BORDER>(v, g, t - 1);
    fine_update<(TT + kWin - 1) % kWin, (TT + kWin - 2) % kWin, TT % kWin, S, EDGE>(v, g);
    fine_update<(TT + kWin - 2) % kWin, (TT + kWin - 3) % kWin, (TT + kWin - 1) % kWin, S, EDGE>(v, g);
    fine_update<(TT + kWin - 3) % kWin, (TT + kWin - 4) % kWin, (TT + kWin - 2) % kWin, S, EDGE>(v, g);
    fine_update<(TT + kWin - 4) % kWin, (TT + kWin - 5) % kWin, (TT + kWin - 3) % kWin, S, EDGE>(v, g);
    if (ST == kStCore || (ST == kStCheck && t - 4 >= g.y0 && t - 4 < g.y1))
        fine_store_row<(TT + kWin - 4) % kWin, PAIR, T>(v, g, t - 4);
    // keep the scheduler from interleaving consecutive steps, which only raises register pressure
    __builtin_amdgcn_sched_barrier(0);
}

template <bool EDGE, bool BORDER, int PAIR, typename T, int ST, bool EN>
__device__ __forceinline__ void fine_block(FineWin &v, const FineGeo &g, RowMap &mi, RowMap &mp,
                                           int t) {
    fine_step<0, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t);
    fine_step<1, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 1);
    fine_step<2, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 2);
    fine_step<3, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 3);
    fine_step<4, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 4);
    fine_step<5, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 5);
    fine_step<6, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 6);
    fine_step<7, EDGE, BORDER, PAIR, T, ST, EN>(v, g, mi, mp, t + 7);
}

// Returns the lane's share of the input state's energy (EN), else 0.
template <typename T, bool EDGE, int PAIR, bool EN>
__device__ __forceinline__ double fine_strip(const FineArgs &args, int sx, int sy, int lane) {
    FineGeo g;
    const size_t planeI = static_cast<size_t>(args.W) * args.H * sizeof(T);
    const size_t planeP = static_cast<size_t>(args.wp) * args.hp * sizeof(T);
    const size_t planeO = static_cast<size_t>(args.w) * args.h * sizeof(T);
    g.pI = static_cast<uint32_t>(planeI);
    g.pP = static_cast<uint32_t>(planeP);
    g.pO = static_cast<uint32_t>(planeO);
    g.A = tensor_rsrc(args.A, planeI);
    g.I = tensor_rsrc(args.I, 3 * planeI);
    g.P = tensor_rsrc(args.Fp, 6 * planeP);
    g.Fo = tensor_rsrc(args.Fo, 3 * planeO);
    g.Bo = tensor_rsrc(args.Bo, 3 * planeO);
    g.W = args.W;
    g.H = args.H;
    g.wp = args.wp;
    g.hp = args.hp;
    g.w = args.w;
    g.h = args.h;
    g.omega = args.omega;
    g.eps = args.eps;
    const int w = args.w, h = args.h, nx = args.nx;

    // Column geometry.  Strip 0 starts at column 0 and the last strip ends at column w-1;
    // interior strips keep 120 core columns.  EDGE strips (the first, the last, or a single
    // strip) contain an image border and resolve it with per-lane selects.
    int xs, cx0, cx1;
    if (nx == 1) {
        xs = 0;
        cx0 = 0;
        cx1 = w;
    } else if (sx == 0) {
        xs = 0;
        cx0 = 0;
        cx1 = kFirstCore;
    } else if (sx == nx - 1) {
        xs = w - kStripCols;
        cx0 = kFirstCore + kMidCore * (nx - 2);
        cx1 = w;
    } else {
        cx0 = kFirstCore + kMidCore * (sx - 1);
        xs = cx0 - kHalo;
        cx1 = cx0 + kMidCore;
    }
    const int xa = xs + 2 * lane, xb = xa + 1;
    const int xa_c = min(xa, w - 1), xb_c = min(xb, w - 1);
    g.sia = static_cast<uint32_t>(xa_c * args.W / w) * sizeof(T);
    g.sib = static_cast<uint32_t>(xb_c * args.W / w) * sizeof(T);
    g.spa = static_cast<uint32_t>(xa_c * args.wp / w) * sizeof(T);
    g.spb = static_cast<uint32_t>(xb_c * args.wp / w) * sizeof(T);
    g.oxa = static_cast<uint32_t>(xa) * sizeof(T);
    g.oxb = static_cast<uint32_t>(xb) * sizeof(T);
    g.store_a = xa >= cx0 && xa < cx1;
    g.store_b = xb >= cx0 && xb < cx1;
    g.left_a = xa == 0;
    g.right_a = xa == w - 1;
    g.right_b = xb == w - 1;

    // Row geometry.  Core rows [y0, y1).  The pipeline starts kHalo rows above y0 (one more when
    // needed so that (xs + t0) is even, which makes the updated column of the pair a
    // compile-time function of t - t0) and ends when row y1-1 is final, at t = y1 - 1 + kNHS.
    // A row's first neighbour outside the processed range is stale, and each half-sweep spreads
    // that by one row, so kHalo rows suffice on each side.
    g.y0 = sy * args.strip_rows;
    g.y1 = min(h, g.y0 + args.strip_rows);
    g.t0 = g.y0 - kHalo - ((xs + g.y0 - kHalo) & 1);
    g.tlast = g.y1 - 1 + kNHS;

    FineWin v;
    v.energy = 0.0;
#pragma unroll
    for (int r = 0; r < kWin; ++r)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            v.ra[r][s] = 0;
            v.al[r][s] = 0.0f;
            v.wl[r][s] = v.wr[r][s] = v.wu[r][s] = v.wd[r][s] = v.ka[r][s] = v.kb[r][s] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v.ri[r][s][c] = v.rf[r][s][c] = v.rb[r][s][c] = 0;
                v.iv[r][s][c] = v.fv[r][s][c] = v.bv[r][s][c] = 0.0f;
            }
        }
    // Row maps for the clamped rows t0, t0+1, ...: input row and previous-level row.
    RowMap mi, mp;
    const int tc0 = min(max(g.t0, 0), h - 1);
    mi.init(tc0, args.H, h);
    mp.init(tc0, args.hp, h);
    fine_load_row<0, PAIR, T>(v, g, mi.q, mp.q);
    static_assert(kPD == 2, "the prologue loads rows t0 and t0 + 1");
    if (g.t0 + 1 >= 1 && g.t0 + 1 <= h - 1) {
        mi.advance();
        mp.advance();
    }
    fine_load_row<1, PAIR, T>(v, g, mi.q, mp.q);

    // Phantom rows -1 and h get their weights at steps 0 and h + 1.  Only the blocks holding
    // those steps use the border variant: a first block with t0 <= 0 or t0 + kWin > h + 1, and
    // the blocks from the one holding step h + 1 on.  The first block stores nothing (its rows
    // t0 - 4 .. t0 + 3 lie above y0, as t0 <= y0 - kHalo); the blocks whose eight stored rows
    // (t - 4 .. t + 3) all lie in the core store without a test.  The regions run one after the
    // other (not as alternatives inside one loop), which keeps the register allocation of the
    // steady state free of spills.  A strip has at least kHalo + 1 + kNHS > kWin steps, so the
    // first block is never its last.
    //
    // The common strip -- no image border, no parity row, whole blocks, at least three -- runs
    // straight through: a first block without stores, then blocks that all store (rows
    // y0 .. y1 - 1 exactly), the last one outside the loop.  (Measured at 4096x3072: the
    // finest level 155 -> 149 us in float32, 95 -> 89 us in float16, against one loop with a
    // store test in every step; the general regions below alone reach 153 / 91 us.)
    int t = g.t0;
    const int nsteps = g.tlast - g.t0 + 1;
    if (t > 0 && g.y0 - t == kHalo && (nsteps & (kWin - 1)) == 0 && nsteps >= 3 * kWin &&
        t + nsteps <= h + 1) {
        fine_block<EDGE, false, PAIR, T, kStNone, EN>(v, g, mi, mp, t);
        for (t += kWin; t + kWin <= g.tlast; t += kWin)
            fine_block<EDGE, false, PAIR, T, kStCore, EN>(v, g, mi, mp, t);
        fine_block<EDGE, false, PAIR, T, kStCore, EN>(v, g, mi, mp, t);
        return v.energy;
    }
    if (t <= 0 || t + kWin > h + 1)
        fine_block<EDGE, true, PAIR, T, kStNone, EN>(v, g, mi, mp, t);
    else
        fine_block<EDGE, false, PAIR, T, kStNone, EN>(v, g, mi, mp, t);
    t += kWin;
    for (; t <= g.tlast && t + kWin <= h + 1 && t - 4 < g.y0; t += kWin)
        fine_block<EDGE, false, PAIR, T, kStCheck, EN>(v, g, mi, mp, t);
    for (; t <= g.tlast && t + kWin <= h + 1 && t + 3 < g.y1; t += kWin)
        fine_block<EDGE, false, PAIR, T, kStCore, EN>(v, g, mi, mp, t);
    for (; t <= g.tlast && t + kWin <= h + 1; t += kWin) fine_block<EDGE, false, PAIR, T, kStCheck, EN>(v, g, mi, mp, t);
    for (; t <= g.tlast; t += kWin) fine_block<EDGE, true, PAIR, T, kStCheck, EN>(v, g, mi, mp, t);
    return v.energy;
}

template <typename T, bool EN = false>
__device__ __forceinline__ double fine_body(const FineArgs &args, int wave, int lane) {
    const int sx = wave % args.nx, sy = wave / args.nx;
    // Paired access needs the identity input map in x; sharing the previous level's column needs
    // the previous level exactly half as wide.  Interior strips start on even columns and keep
    // even core boundaries at any width, so a lane's two columns are both stored or both not;
    // in an odd-width level the pair of an odd row starts at an odd element, an access aligned
    // to its element size only, which the vector-memory path performs as an unaligned access.
    // Of the two border strips of a level wider than one strip, the first starts at column 0
    // and qualifies at any width; the last ends at column w - 1, so it starts on an even column
    // only when w is even.  The border clamp is a per-lane select either way.  A level of one
    // strip (w <= 128) has lanes past the last column and stays unpaired.
    const bool pair_in = args.w == args.W && args.w > kStripCols;
    const bool pair_full = pair_in && 2 * args.wp == args.w;
    const bool pair_same = pair_in && args.wp == args.w;   // instantiated for the energy kernel
    if (args.w <= kStripCols || sx == 0 || sx == args.nx - 1) {
        const bool edge_ok = sx == 0 || (args.w & 1) == 0;
        if constexpr (EN)
            if (edge_ok && pair_same) return fine_strip<T, true, kPairSame, EN>(args, sx, sy, lane);
        if (edge_ok && pair_full)
            return fine_strip<T, true, kPairFull, EN>(args, sx, sy, lane);
        else if (edge_ok && pair_in)
            return fine_strip<T, true, kPairIn, EN>(args, sx, sy, lane);
        else
            return fine_strip<T, true, kPairNone, EN>(args, sx, sy, lane);
    } else if (EN && pair_same) {
        return fine_strip<T, false, EN ? kPairSame : kPairIn, EN>(args, sx, sy, lane);
    } else if (pair_full) {
        return fine_strip<T, false, kPairFull, EN>(args, sx, sy, lane);
    } else if (pair_in) {
        return fine_strip<T, false, kPairIn, EN>(args, sx, sy, lane);
    } else {
        return fine_strip<T, false, kPairNone, EN>(args, sx, sy, lane);
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b on XCD b % 8), each with its
// own L2.  The row-major sequence of blocks (kWavesPerBlock strips each) is cut into 8 equal
// chunks and chunk c runs on XCD c: each XCD then streams a band of whole-width strip rows, and
// vertically adjacent strips, which read each other's halo rows, share an L2.
__host__ __device__ inline int fine_block_chunk(int units) {
    const int blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    return (blocks + kXcds - 1) / kXcds;
}

template <typename T>
__global__ __launch_bounds__(64 * kWavesPerBlock, 2) void fine_kernel(FineArgs args) {
    const int units = args.nx * args.ny;
    const int pos = (blockIdx.x % kXcds) * fine_block_chunk(units) + blockIdx.x / kXcds;
    const int wave = uniform(pos * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= units) return;
    fine_body<T>(args, wave, threadIdx.x & 63);
}

// The convergence form's passes (float32 state): the streaming pass that also reduces the energy
// of the state it starts from, one partial per strip (epart[5 * strip], fge_energy's layout).
__global__ __launch_bounds__(64 * kWavesPerBlock, 2) void fine_energy_kernel(FineArgs args,
                                                                             double *epart,
                                                                             const int *skip) {
    if (skip && *skip) return;   // the level has stopped
    const int units = args.nx * args.ny;
    const int pos = (blockIdx.x % kXcds) * fine_block_chunk(units) + blockIdx.x / kXcds;
    const int wave = uniform(pos * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= units) return;
    double e = fine_body<float, true>(args, wave, threadIdx.x & 63);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0) {
        double *o = epart + 5 * static_cast<size_t>(wave);
        o[0] = e;
        o[1] = o[2] = o[3] = o[4] = 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// Batched, persistent kernels: many images' levels in one launch.
// ------------------------------------------------------------------------------------------
//
// A launch gets a descriptor table (one FineArgs / TileArgs per image level) and a work list of
// (descriptor, unit) items, unit = strip (streaming kernel) or tile (tile kernel).  Waves (or
// workgroups) of a grid sized to the machine pull items from an atomic counter in the workspace
// until the list is exhausted: the per-level work queue.  Every item is processed by the same
// body as the single-image kernels, so a batched image's result is bit-identical to its
// single-image result.  The counters are zeroed by zero_kernel (not a memset), so the schedule
// can be captured in a hipGraph and replayed.


__global__ void zero_kernel(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// A descriptor that every lane of a wave loaded from the same address, with each 32-bit word
// taken from the first active lane.  The compiler then knows every field is wave-uniform, so the
// buffer resources built from the pointers live in scalar registers; a resource it must assume
// may differ across lanes turns every buffer access into a loop over the lanes' distinct values.
template <typename S>
__device__ __forceinline__ S uniform_copy(const S &s) {
    static_assert(sizeof(S) % 4 == 0, "descriptor of whole 32-bit words");
    int words[sizeof(S) / 4];
    __builtin_memcpy(words, &s, sizeof(S));
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(S) / 4); ++i)
        words[i] = __builtin_amdgcn_readfirstlane(words[i]);
    S r;
    __builtin_memcpy(&r, words, sizeof(S));
    return r;
}

// One item per wave.  The counter is bumped by lane 0 with a vector atomic and broadcast.
__device__ __forceinline__ int next_item_wave(int *counter, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(counter, 1);
    return uniform(__shfl(v, 0));
}

// Per-XCD work queues.  Workgroup b runs on XCD b % 8; the launch's item list is cut into chunks
// of kQueueChunk consecutive items (a few bands of neighbouring strips of one image) and chunk j
// belongs to XCD j % 8, whose waves take its items in order from the XCD's own counter.  Strips
// that share halo rows and the cache lines at their column boundaries then mostly run at the
// same time on one XCD and meet in its L2, instead of being fetched once per XCD.  Chunks of all
// images are dealt round-robin, so the XCDs' loads differ by at most about a chunk.  Used for
// launches of at least two rounds of waves (kXcdQueueMinItems); smaller launches take items from
// one shared counter (measured: a one-round launch ran ~10% slower on per-XCD queues, and the
// LDS tile launches, with their larger work units, ~25% slower).
constexpr int kQueueChunk = 64;

__device__ __forceinline__ int next_item_xcd(int *counters, int xcd, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(counters + xcd, 1);
    v = uniform(__shfl(v, 0));
    const int chunk = v / kQueueChunk;
    return (chunk * kXcds + xcd) * kQueueChunk + (v - chunk * kQueueChunk);
}

template <typename T>
__global__ __launch_bounds__(64 * kWavesPerBlock, 2) void fine_batch_kernel(
    const FineArgs *descs, const WorkItem *items, int nitems, int *counters, int per_xcd) {
    const int lane = threadIdx.x & 63;
    const int xcd = blockIdx.x % kXcds;
    for (;;) {
        const int it = per_xcd ? next_item_xcd(counters, xcd, lane) : next_item_wave(counters, lane);
        if (it >= nitems) return;
        const WorkItem w = items[it];
        const FineArgs a = uniform_copy(descs[uniform(w.desc)]);
        fine_body<T>(a, uniform(w.unit), lane);
    }
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void tile_batch_kernel(
    const TileArgs *descs, const WorkItem *items, int nitems, int *counters) {
    __shared__ TileLds lds;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counters, 1);
        lds_sync();
        const int it = s_item;
        lds_sync();   // everyone has read s_item (and the previous tile is stored)
        if (it >= nitems) return;
        const WorkItem w = items[it];
        tile_body<T>(descs[w.desc], w.unit, lds);
        lds_sync();   // the tile's LDS is free for the next item
    }
}

// Gather pre-pass: unit p writes pixel p of the concatenated small levels of one image: I (3
// planes) and alpha resized from full resolution by the nearest map, into each level's compact
// planes.
// One pixel of a gather: the four values read, and where they go.
template <typename T>
struct GatherPx {
    T *dst;
    size_t n;
    int q;
    T v[4];
};

template <typename T>
__device__ __forceinline__ void gather_fetch(const GatherArgs &args, long long p, GatherPx<T> &g) {
    int l = 0;
    while (l + 1 < args.ng && p >= args.first[l + 1]) ++l;
    const int w = args.lw[l], h = args.lh[l];
    const int q = static_cast<int>(p - args.first[l]);
    const float rw = rcp(static_cast<float>(w)), rh = rcp(static_cast<float>(h));
    const int y = fdiv(q, w, rw), x = q - y * w;
    const size_t planeI = static_cast<size_t>(args.W) * args.H;
    const size_t src = static_cast<size_t>(fdiv(y * args.H, h, rh)) * args.W + fdiv(x * args.W, w, rw);
    const T *I = static_cast<const T *>(args.I);
    g.dst = reinterpret_cast<T *>(args.pyr + args.off[l]);
    g.n = static_cast<size_t>(w) * h;
    g.q = q;
#pragma unroll
    for (int c = 0; c < 3; ++c) g.v[c] = I[c * planeI + src];
    g.v[3] = static_cast<const T *>(args.A)[src];
}

template <typename T>
__device__ __forceinline__ void gather_put(const GatherPx<T> &g) {
#pragma unroll
    for (int c = 0; c < 4; ++c) g.dst[c * g.n + g.q] = g.v[c];
}

template <typename T>
__device__ __forceinline__ void gather_body(const GatherArgs &args, long long p) {
    GatherPx<T> g;
    gather_fetch<T>(args, p, g);
    gather_put<T>(g);
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs args) {
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < args.first[args.ng]) gather_body<T>(args, p);
}

// The coarse block and the gather of the levels after it in one launch.  Workgroup 0 runs the
// coarse levels (their inputs come from full resolution); the others copy the compact inputs of
// the later levels, grid-stride, kGatherUnroll pixels per thread in flight at once.  The levels
// that read those copies run in later launches.
constexpr int kGatherUnroll = 16;
constexpr int kGatherBlocksMax = 255;   // every CU but the coarse block's

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void coarse_gather_kernel(CoarseArgs cargs,
                                                                       GatherArgs gargs) {
    __shared__ CoarseLds lds;
    if (blockIdx.x == 0) {
        coarse_body<T>(cargs, lds);
        return;
    }
    const long long total = gargs.first[gargs.ng];
    const long long stride = static_cast<long long>(gridDim.x - 1) * kCoarseThreads;
    for (long long base = static_cast<long long>(blockIdx.x - 1) * kCoarseThreads + threadIdx.x;
         base < total; base += stride * kGatherUnroll) {
        GatherPx<T> g[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {   // every load first ...
            const long long p = base + u * stride;
            if (p < total) gather_fetch<T>(gargs, p, g[u]);
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u)      // ... then the stores
            if (base + u * stride < total) gather_put<T>(g[u]);
    }
}

// Batch: `first` holds each image's first pixel in the concatenation of all images' gathers.
template <typename T>
__global__ __launch_bounds__(256) void gather_batch_kernel(const GatherArgs *descs,
                                                           const long long *first, int n,
                                                           long long total) {
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= total) return;
    int lo = 0, hi = n - 1;   // last image whose first pixel is <= p
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= p) lo = mid; else hi = mid - 1;
    }
    gather_body<T>(descs[lo], p - first[lo]);
}

int auto_strip_rows(int w, int h) {
    // The height that gives one round of two waves per SIMD (256 CUs x 4 SIMDs x 2), so one
    // wave's memory waits overlap the other's arithmetic, clamped to [8, 16] rows.  Measured at
    // 4096x3072 over 6..64 rows: levels whose round would need taller strips run faster as
    // several rounds of 16-row strips (the XCD-chunked block order then keeps each XCD's
    // resident strips within a band of ~120 rows, whose shared halo rows hit in its L2) in spite
    // of the larger halo share; below 8 rows the halo (9 extra rows per strip) dominates.
    const long nx = fine_strips_x(w);
    const long two = (static_cast<long>(h) * nx + 2047) / 2048;
    long rows = two < 8 ? 8 : (two > 16 ? 16 : two);
    rows = (rows + 1) & ~1L;
    if (rows > h) rows = h;
    return static_cast<int>(rows);
}

template <typename T>
int launch_naive_t(const LevelIO &io, int iters, hipStream_t s) {
    const int n = io.w * io.h;
    hipLaunchKernelGGL(upsample_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, s,
                       static_cast<const T *>(io.Fp), static_cast<const T *>(io.Bp), io.wp, io.hp,
                       static_cast<T *>(io.Fo), static_cast<T *>(io.Bo), io.w, io.h);
    int err = static_cast<int>(hipGetLastError());
    if (err) return err;
    const int npairs = ((io.w + 1) / 2) * io.h;
    for (int it = 0; it < iters; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
            hipLaunchKernelGGL(halfsweep_kernel<T>, dim3((npairs + 255) / 256), dim3(256), 0, s,
                               static_cast<const T *>(io.I), static_cast<const T *>(io.A), io.W,
                               io.H, static_cast<T *>(io.Fo), static_cast<T *>(io.Bo), io.w, io.h,
                               colour, io.omega, io.eps);
            err = static_cast<int>(hipGetLastError());
            if (err) return err;
        }
    }
    return 0;
}

// Persistent grids: enough waves / workgroups to fill the machine, never more than the items.
constexpr int kPersistentWaves = 256 * 4 * 2;      // two waves per SIMD
constexpr int kXcdQueueMinItems = 2 * kPersistentWaves;   // per-XCD queues from two rounds on
constexpr int kPersistentTileGroups = 256 * 2;     // two tile workgroups per CU

}  // namespace

// ---- descriptor builders ----------------------------------------------------------------

void make_fine_args(const LevelIO &io, int strip_rows, FineArgs *a) {
    *a = FineArgs{};
    a->I = io.I;
    a->A = io.A;
    a->W = io.W;
    a->H = io.H;
    a->Fp = io.Fp;
    a->Bp = io.Bp;
    a->wp = io.wp;
    a->hp = io.hp;
    a->Fo = io.Fo;
    a->Bo = io.Bo;
    a->w = io.w;
    a->h = io.h;
    a->omega = io.omega;
    a->eps = io.eps;
    a->nx = fine_strips_x(io.w);
    a->strip_rows = strip_rows > 0 ? strip_rows : auto_strip_rows(io.w, io.h);
    a->ny = (io.h + a->strip_rows - 1) / a->strip_rows;
}

int fine_units(const FineArgs &a) { return a.nx * a.ny; }

int launch_strip_rows(const int *w, const int *h, int n) {
    // A batched launch has the parallelism of all its levels together, so its strips can be
    // taller than one level alone would get (less halo work per output row): the tallest even
    // height up to 32 rows that still gives every resident wave a strip.  Taller strips lose
    // again (64 uneven images, float16, per batch: 1.58 ms at 24-32 rows, 1.62 ms at 48 and 64,
    // 1.60 ms at 16).
    for (int rows = 32; rows >= 8; rows -= 2) {
        long items = 0;
        for (int k = 0; k < n; ++k)
            items += static_cast<long>(fine_strips_x(w[k])) * ((h[k] + rows - 1) / rows);
        if (items >= kPersistentWaves) return rows;
    }
    return 0;
}

void make_tile_args(const LevelIO &io, TileArgs *a) {
    *a = TileArgs{};
    a->I = io.I;
    a->A = io.A;
    a->W = io.W;
    a->H = io.H;
    a->Fp = io.Fp;
    a->Bp = io.Bp;
    a->wp = io.wp;
    a->hp = io.hp;
    a->Fo = io.Fo;
    a->Bo = io.Bo;
    a->w = io.w;
    a->h = io.h;
    a->omega = io.omega;
    a->eps = io.eps;
    a->tiles_x = (io.w + kTileCore - 1) / kTileCore;
}

int tile_units(const TileArgs &a) { return a.tiles_x * ((a.h + kTileCore - 1) / kTileCore); }

void make_coarse_args(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                      float eps, CoarseArgs *a) {
    *a = CoarseArgs{};
    a->src = src;
    a->Fo = Fo;
    a->Bo = Bo;
    a->nc = plan.nc;
    for (int i = 0; i < plan.nc; ++i) {
        a->lw[i] = plan.lv[i].w;
        a->lh[i] = plan.lv[i].h;
        a->lit[i] = plan.lv[i].iters;
    }
    a->omega = omega;
    a->eps = eps;
}

void make_gather_args(const Plan &plan, const void *I, const void *A, void *pyr, GatherArgs *a) {
    *a = GatherArgs{};
    a->I = I;
    a->A = A;
    a->W = plan.W;
    a->H = plan.H;
    a->pyr = static_cast<char *>(pyr);
    a->ng = plan.ng;
    long long total = 0;
    for (int i = 0, k = 0; i < plan.n; ++i) {
        if (!plan.copy[i]) continue;
        a->lw[k] = plan.lv[i].w;
        a->lh[k] = plan.lv[i].h;
        a->first[k] = total;
        a->off[k] = static_cast<long long>(plan.pyr_lv[i]);
        total += static_cast<long long>(plan.lv[i].w) * plan.lv[i].h;
        ++k;
    }
    a->first[plan.ng] = total;
}

long long gather_units(const GatherArgs &a) { return a.first[a.ng]; }

// ---- single-image launches --------------------------------------------------------------

#define FGE_DISPATCH(storage, KERNEL, ...)                                                    \
    do {                                                                                      \
        if ((storage) == FGE_F16)                                                             \
            hipLaunchKernelGGL(KERNEL<_Float16>, __VA_ARGS__);                                \
        else                                                                                  \
            hipLaunchKernelGGL(KERNEL<float>, __VA_ARGS__);                                   \
    } while (0)

int launch_gather(const Plan &plan, const void *I, const void *A, void *pyr, int storage,
                  void *stream) {
    GatherArgs a;
    make_gather_args(plan, I, A, pyr, &a);
    const int blocks = static_cast<int>((gather_units(a) + 255) / 256);
    FGE_DISPATCH(storage, gather_kernel, dim3(blocks), dim3(256), 0,
                 static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_coarse_gather(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                         float eps, const void *I, const void *A, void *pyr, int storage,
                         void *stream) {
    CoarseArgs c;
    make_coarse_args(plan, src, Fo, Bo, omega, eps, &c);
    GatherArgs g;
    make_gather_args(plan, I, A, pyr, &g);
    const long long per_block = static_cast<long long>(kCoarseThreads) * kGatherUnroll;
    const long long want = (gather_units(g) + per_block - 1) / per_block;
    const int gblocks = static_cast<int>(want < kGatherBlocksMax ? want : kGatherBlocksMax);
    FGE_DISPATCH(storage, coarse_gather_kernel, dim3(1 + gblocks), dim3(kCoarseThreads), 0,
                 static_cast<hipStream_t>(stream), c, g);
    return static_cast<int>(hipGetLastError());
}

int launch_coarse(const Plan &plan, const LevelSrc &src, void *Fo, void *Bo, float omega,
                  float eps, int storage, void *stream) {
    CoarseArgs a;
    make_coarse_args(plan, src, Fo, Bo, omega, eps, &a);
    FGE_DISPATCH(storage, coarse_kernel, dim3(1), dim3(kCoarseThreads), 0,
                 static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_coarse_converge(const CoarseArgs &a, double tol, int max_passes, int *counts,
                           void *stream) {
    hipLaunchKernelGGL(coarse_conv_kernel, dim3(1), dim3(kCoarseThreads), 0,
                       static_cast<hipStream_t>(stream), a, tol, max_passes, counts);
    return static_cast<int>(hipGetLastError());
}

int launch_fine_fused(const LevelIO &io, int strip_rows, int storage, void *stream) {
    FineArgs a;
    make_fine_args(io, strip_rows, &a);
    const int blocks = kXcds * fine_block_chunk(fine_units(a));
    FGE_DISPATCH(storage, fine_kernel, dim3(blocks), dim3(64 * kWavesPerBlock), 0,
                 static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

void make_pyramid_args(const Plan &plan, char *ws, const void *I, const void *A, void *F,
                       void *B, float omega, float eps, int first, int last, PyramidArgs *a) {
    *a = PyramidArgs{};
    a->nl = last - first + 1;
    for (int j = first; j <= last; ++j) {
        const LevelIO io = level_io(plan, ws, j, I, A, F, B, omega, eps);
        PyramidLevel &d = a->lv[j - first];
        d.I = io.I;
        d.A = io.A;
        d.W = io.W;
        d.H = io.H;
        d.w = io.w;
        d.h = io.h;
        if (j == first) {
            a->Fp = io.Fp;
            a->Bp = io.Bp;
            a->wp = io.wp;
            a->hp = io.hp;
        }
        if (j == last) {
            a->Fo = io.Fo;
            a->Bo = io.Bo;
            a->tiles_x = (io.w + kTileCore - 1) / kTileCore;
            a->tiles = a->tiles_x * ((io.h + kTileCore - 1) / kTileCore);
        }
    }
    a->omega = omega;
    a->eps = eps;
}

bool pyramid_fits(const Plan &plan, int first, int last) {
    if (first < 1 || last <= first || last - first + 1 > kPyrMaxLevels) return false;
    PyramidArgs a{};
    a.nl = last - first + 1;
    for (int j = first; j <= last; ++j) {
        a.lv[j - first].w = plan.lv[j].w;
        a.lv[j - first].h = plan.lv[j].h;
    }
    a.tiles_x = (plan.lv[last].w + kTileCore - 1) / kTileCore;
    const int tiles = a.tiles_x * ((plan.lv[last].h + kTileCore - 1) / kTileCore);
    TileRegion R[kPyrMaxLevels];
    for (int t = 0; t < tiles; ++t) {
        pyramid_regions(a, t, R);
        for (int l = 0; l < a.nl; ++l)
            if (R[l].rw > kTileSide || R[l].rh > kTileSide || R[l].rw < 1 || R[l].rh < 1) return false;
    }
    return true;
}

int launch_pyramid(const Plan &plan, char *ws, const void *I, const void *A, void *F, void *B,
                   float omega, float eps, int storage, void *stream) {
    PyramidArgs a;
    make_pyramid_args(plan, ws, I, A, F, B, omega, eps, plan.pyr_first, plan.pyr_last, &a);
    FGE_DISPATCH(storage, pyramid_kernel, dim3(a.tiles), dim3(kTileThreads), 0,
                 static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_fine_tile(const LevelIO &io, int storage, void *stream) {
    TileArgs a;
    make_tile_args(io, &a);
    FGE_DISPATCH(storage, tile_kernel, dim3(tile_units(a)), dim3(kTileThreads), 0,
                 static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int pass_energy_parts(const LevelIO &io, int strip_rows, bool tile) {
    if (tile) {
        TileArgs a;
        make_tile_args(io, &a);
        return tile_units(a);
    }
    FineArgs a;
    make_fine_args(io, strip_rows, &a);
    return fine_units(a);
}

int launch_pass_energy(const LevelIO &io, int strip_rows, bool tile, double *epart,
                       const int *skip, void *stream, bool jacobi) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (tile || jacobi) {
        TileArgs a;
        make_tile_args(io, &a);
        if (jacobi)
            hipLaunchKernelGGL(tile_energy_kernel<true>, dim3(tile_units(a)), dim3(kTileThreads), 0, s,
                               a, epart, skip);
        else
            hipLaunchKernelGGL(tile_energy_kernel<false>, dim3(tile_units(a)), dim3(kTileThreads), 0,
                               s, a, epart, skip);
    } else {
        FineArgs a;
        make_fine_args(io, strip_rows, &a);
        const int blocks = kXcds * fine_block_chunk(fine_units(a));
        hipLaunchKernelGGL(fine_energy_kernel, dim3(blocks), dim3(64 * kWavesPerBlock), 0, s, a,
                           epart, skip);
    }
    return static_cast<int>(hipGetLastError());
}

int launch_naive_level(const LevelIO &io, int iters, int storage, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (storage == FGE_F16) return launch_naive_t<_Float16>(io, iters, s);
    return launch_naive_t<float>(io, iters, s);
}

// ---- batched launches -------------------------------------------------------------------

int launch_zero(int *d, int n, void *stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), d, n);
    return static_cast<int>(hipGetLastError());
}

int launch_gather_batch(const GatherArgs *descs, const long long *first, int n, long long total,
                        int storage, void *stream) {
    if (total <= 0) return 0;
    const int blocks = static_cast<int>((total + 255) / 256);
    FGE_DISPATCH(storage, gather_batch_kernel, dim3(blocks), dim3(256), 0,
                 static_cast<hipStream_t>(stream), descs, first, n, total);
    return static_cast<int>(hipGetLastError());
}

int launch_coarse_batch(const CoarseArgs *descs, int n, int storage, void *stream) {
    if (n <= 0) return 0;
    FGE_DISPATCH(storage, coarse_batch_kernel, dim3(n), dim3(kCoarseThreads), 0,
                 static_cast<hipStream_t>(stream), descs);
    return static_cast<int>(hipGetLastError());
}

int launch_fine_batch(const FineArgs *descs, const WorkItem *items, int nitems, int *counter,
                      int storage, void *stream) {
    if (nitems <= 0) return 0;
    const int waves = nitems < kPersistentWaves ? nitems : kPersistentWaves;
    const int blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;   // a multiple of 8 when
    const int per_xcd = nitems >= kXcdQueueMinItems ? 1 : 0;            // per_xcd (2048 waves)
    FGE_DISPATCH(storage, fine_batch_kernel, dim3(blocks), dim3(64 * kWavesPerBlock), 0,
                 static_cast<hipStream_t>(stream), descs, items, nitems, counter, per_xcd);
    return static_cast<int>(hipGetLastError());
}

int launch_tile_batch(const TileArgs *descs, const WorkItem *items, int nitems, int *counter,
                      int storage, void *stream) {
    if (nitems <= 0) return 0;
    const int groups = nitems < kPersistentTileGroups ? nitems : kPersistentTileGroups;
    FGE_DISPATCH(storage, tile_batch_kernel, dim3(groups), dim3(kTileThreads), 0,
                 static_cast<hipStream_t>(stream), descs, items, nitems, counter);
    return static_cast<int>(hipGetLastError());
}

}  // namespace fge
