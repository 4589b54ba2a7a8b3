// The level loop of Algorithm 1 in its "while not converged" form, and the Jacobi sweep order,
// on the device (C ABI in include/fge.h).
//
// Per level: resize F and B from the previous level (nearest), then sweep.  With a tolerance
// tol >= 0 the level's energy (fge_energy's quadratic on the level's F, B against its resized
// image and matte) is reduced on the device after every sweep, and the launch that totals it
// compares it with the energy before the sweep: when |E_prev - E| <= tol E_prev, or after
// max_sweeps sweeps, it raises a stop flag that turns every later launch of the level into a
// no-op (grid-stride kernels with capped grids, so a stopped launch retires quickly).  The host
// enqueues max_sweeps guarded sweeps without waiting; the decision never leaves the device.
// With tol < 0 every level runs the fixed counts of the iteration rule (10 / 2), unguarded.
//
// Resize variants: nearest (Algorithm 1 as read everywhere else) or smooth (the image and matte
// area-averaged from full resolution into float32 level copies, the previous level's F and B
// resized bilinearly).  The smooth variant with the red-black order and fixed counts sweeps on
// the fused kernels (cv_fused_sweeps).
//
// Orders: red-black (two half-sweeps in place, (x + y) even first) or Jacobi (every pixel from
// the previous sweep's values: sweeps alternate between two buffers, the result copied back
// once at the end of the level if it ran an odd number).  The per-pixel update is the
// 2x2 solve of eq. 9 in the same Sherman-Morrison form as the other kernels.  A level sweeps on
// float32 working buffers and its state is converted to the storage type once, when the level is
// written (so binary16 storage rounds once per level, as on the fused path).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>

#include "fge_internal.h"

namespace fge {
namespace {

constexpr int kCvThreads = 256;
constexpr int kCvBlocksMax = 4096;
constexpr int kCvMaxSweeps = 100000;

template <typename T>
__device__ __forceinline__ float ldv(const T *p, size_t i) { return static_cast<float>(p[i]); }
template <typename T>
__device__ __forceinline__ void stv(T *p, size_t i, float v) { p[i] = static_cast<T>(v); }
__device__ __forceinline__ float clamp_unit(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }
__device__ __forceinline__ bool stopped(const int *stop) { return stop && *stop; }

unsigned blocks_for(size_t n) {
    const size_t b = (n + kCvThreads - 1) / kCvThreads;
    return static_cast<unsigned>(b < static_cast<size_t>(kCvBlocksMax) ? b : kCvBlocksMax);
}

template <typename T>
__global__ __launch_bounds__(kCvThreads) void cv_upsample_kernel(const T *Fp, const T *Bp, int wp,
                                                                 int hp, float *Fo, float *Bo, int w,
                                                                 int h) {
    const size_t n = static_cast<size_t>(w) * h, np = static_cast<size_t>(wp) * hp;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<size_t>(y) * w);
        const size_t q = static_cast<size_t>(y * hp / h) * wp + x * wp / w;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            stv(Fo, c * n + p, Fp ? ldv(Fp, c * np + q) : 0.0f);
            stv(Bo, c * n + p, Bp ? ldv(Bp, c * np + q) : 0.0f);
        }
    }
}

// Bilinear resize of the previous level's F and B (smooth variant): pixel centres at half-integers,
// source coordinate (x + 1/2) wp / w - 1/2 clamped to [0, wp - 1], likewise in y.
template <typename T>
__global__ __launch_bounds__(kCvThreads) void cv_bilinear_kernel(const T *Fp, const T *Bp, int wp,
                                                                 int hp, float *Fo, float *Bo, int w,
                                                                 int h) {
    const size_t n = static_cast<size_t>(w) * h, np = static_cast<size_t>(wp) * hp;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<size_t>(y) * w);
        auto tap = [](int i, int ns, int nd, int *i0, int *i1, double *f) {
            double u = (i + 0.5) * ns / nd - 0.5;
            u = u < 0.0 ? 0.0 : (u > ns - 1 ? ns - 1 : u);
            *i0 = static_cast<int>(u);
            *i1 = *i0 + 1 < ns ? *i0 + 1 : ns - 1;
            *f = u - *i0;
        };
        int x0, x1, y0, y1;
        double fx, fy;
        tap(x, wp, w, &x0, &x1, &fx);
        tap(y, hp, h, &y0, &y1, &fy);
        auto mix = [&](const T *P) {
            const double top = (1.0 - fx) * static_cast<float>(P[static_cast<size_t>(y0) * wp + x0]) +
                               fx * static_cast<float>(P[static_cast<size_t>(y0) * wp + x1]);
            const double bot = (1.0 - fx) * static_cast<float>(P[static_cast<size_t>(y1) * wp + x0]) +
                               fx * static_cast<float>(P[static_cast<size_t>(y1) * wp + x1]);
            return static_cast<float>((1.0 - fy) * top + fy * bot);
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Fo[c * n + p] = Fp ? mix(Fp + c * np) : 0.0f;
            Bo[c * n + p] = Bp ? mix(Bp + c * np) : 0.0f;
        }
    }
}

// Area resize (smooth variant), separable: destination pixel u of an axis of nd pixels averages
// the source over [u ns/nd, (u+1) ns/nd), every source pixel weighted by its overlap.  Pass 1
// (ROWS) resizes the rows of the 4 input planes (I then alpha, W x H, type T) to w columns; pass 2
// the columns of that result (float32) to h rows.  Sums in float64, results in float32.  A launch
// is a grid of (destination pixels of a row, rows, 4 planes); G lanes (a power of two up to 64,
// about an eighth of the footprint's length) share one destination pixel: lane g takes source
// pixels i0 + g, i0 + g + G, ..., and the group adds its partial sums in a fixed butterfly.  The
// footprint's ends are u times the float64 quotient ns / nd (within a few ulps of u ns / nd; an
// end that lands a rounding off an integer only adds or drops a pixel of weight ~1e-16).
__device__ __forceinline__ double area_span(int u, double step, int ns, int *i0, int *i1,
                                            double *x0, double *x1) {
    *x0 = static_cast<double>(u) * step;
    *x1 = static_cast<double>(u + 1) * step;
    *i0 = static_cast<int>(floor(*x0));
    *i1 = static_cast<int>(ceil(*x1));
    if (*i1 > ns) *i1 = ns;
    return *x1 - *x0;
}

// log2 of the lanes per destination pixel for a footprint of ns / nd source pixels.
int area_group_log2(int ns, int nd) {
    const int f = (ns + nd - 1) / nd;
    int lg = 0;
    while ((8 << lg) < f && lg < 6) ++lg;
    return lg;
}

// ROWS: I (3 planes) and A, W x H, into 4 planes of w x H.  Columns: I = the rows pass's output
// (4 planes of w x H, float32), into 4 planes of w x h.  step = ns / nd of the resized axis.
template <typename T, bool ROWS>
__global__ __launch_bounds__(kCvThreads) void cv_area_kernel(const T *I, const T *A, int W, int H,
                                                             int w, int h, int lg, double step,
                                                             float *out) {
    const int G = 1 << lg;
    const int c = blockIdx.z, y = blockIdx.y;
    const int t = blockIdx.x * kCvThreads + threadIdx.x;
    const int x = t >> lg, g = t & (G - 1);
    if (x >= w) return;   // whole groups: G divides the block
    int i0, i1;
    double x0, x1;
    const double len = ROWS ? area_span(x, step, W, &i0, &i1, &x0, &x1)
                            : area_span(y, step, H, &i0, &i1, &x0, &x1);
    const T *line;
    size_t stride;
    if (ROWS) {
        line = (c < 3 ? I + static_cast<size_t>(c) * W * H : A) + static_cast<size_t>(y) * W;
        stride = 1;
    } else {
        line = I + static_cast<size_t>(c) * w * H + x;
        stride = static_cast<size_t>(w);
    }
    double acc = 0.0;
    for (int i = i0 + g; i < i1; i += G) {
        const double a = i > x0 ? i : x0, b = i + 1 < x1 ? i + 1 : x1;
        acc += (b - a) * static_cast<float>(line[static_cast<size_t>(i) * stride]);
    }
    for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const int ho = ROWS ? H : h;
    if (g == 0) out[(static_cast<size_t>(c) * ho + y) * w + x] = static_cast<float>(acc / len);
}

// The update of pixel (x, y) of a w x h level from the state (F, B), with I and alpha read from
// W x H through the nearest map.
template <typename T>
__device__ __forceinline__ void cv_solve(const T *I, const T *A, int W, int H, const float *F,
                                         const float *B, int w, int h, int x, int y, float omega,
                                         float eps, float fo[3], float bo[3]) {
    const size_t n = static_cast<size_t>(w) * h, nI = static_cast<size_t>(W) * H;
    auto alpha_at = [&](int xx, int yy) {
        return ldv(A, static_cast<size_t>(yy * H / h) * W + xx * W / w);
    };
    const float a = alpha_at(x, y), b = 1.0f - a;
    const int xs[4] = {x > 0 ? x - 1 : 0, x < w - 1 ? x + 1 : w - 1, x, x};
    const int ys[4] = {y, y, y > 0 ? y - 1 : 0, y < h - 1 ? y + 1 : h - 1};
    float s[4], S = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        s[j] = fmaf(omega, fabsf(a - alpha_at(xs[j], ys[j])), eps);
        S += s[j];
    }
    const float iS = 1.0f / S;
    const float k = 1.0f / (S + fmaf(a, a, b * b));
    const size_t src = static_cast<size_t>(y * H / h) * W + x * W / w;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float P = 0.0f, Q = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t nj = c * n + static_cast<size_t>(ys[j]) * w + xs[j];
            P = fmaf(s[j], ldv(F, nj), P);
            Q = fmaf(s[j], ldv(B, nj), Q);
        }
        const float fb = P * iS, bb = Q * iS;
        const float r = ldv(I, c * nI + src) - a * fb - b * bb;
        fo[c] = clamp_unit(fmaf(a * k, r, fb));
        bo[c] = clamp_unit(fmaf(b * k, r, bb));
    }
}

// Red-black half-sweep in place: every pixel with (x + y) % 2 == colour.
template <typename T>
__global__ __launch_bounds__(kCvThreads) void cv_halfsweep_kernel(const T *I, const T *A, int W,
                                                                  int H, float *F, float *B, int w,
                                                                  int h,
                                                                  int colour, float omega,
                                                                  float eps, const int *stop) {
    if (stopped(stop)) return;
    const int pw = (w + 1) >> 1;
    const size_t npairs = static_cast<size_t>(pw) * h, n = static_cast<size_t>(w) * h;
    for (size_t q = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; q < npairs;
         q += static_cast<size_t>(gridDim.x) * kCvThreads) {
        const int y = static_cast<int>(q / pw);
        const int x = 2 * static_cast<int>(q - static_cast<size_t>(y) * pw) + ((y + colour) & 1);
        if (x >= w) continue;
        float fo[3], bo[3];
        cv_solve(I, A, W, H, F, B, w, h, x, y, omega, eps, fo, bo);
        const size_t i = static_cast<size_t>(y) * w + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            stv(F, c * n + i, fo[c]);
            stv(B, c * n + i, bo[c]);
        }
    }
}

// Jacobi sweep: every pixel from the previous state (F, B) into (Fo, Bo).
template <typename T>
__global__ __launch_bounds__(kCvThreads) void cv_jacobi_kernel(const T *I, const T *A, int W, int H,
                                                               const float *F, const float *B,
                                                               float *Fo, float *Bo, int w, int h,
                                                               float omega,
                                                               float eps, const int *stop) {
    if (stopped(stop)) return;
    const size_t n = static_cast<size_t>(w) * h;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<size_t>(y) * w);
        float fo[3], bo[3];
        cv_solve(I, A, W, H, F, B, w, h, x, y, omega, eps, fo, bo);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            stv(Fo, c * n + p, fo[c]);
            stv(Bo, c * n + p, bo[c]);
        }
    }
}

// Copy of the 3 planes of F and of B, converted to the destination type: back from the Jacobi
// temporary (guarded), and the level's working state into its stored state (unguarded).
template <typename TD>
__global__ __launch_bounds__(kCvThreads) void cv_copy_kernel(const float *Fs, const float *Bs,
                                                             TD *F, TD *B, size_t n,
                                                             const int *stop) {
    if (stopped(stop)) return;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < 3 * n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        F[p] = static_cast<TD>(Fs[p]);
        B[p] = static_cast<TD>(Bs[p]);
    }
}

// The Jacobi sweeps of a level alternate between two state buffers; the level's result is in the
// second one when the count of sweeps run is odd: copy it back then.
__global__ __launch_bounds__(kCvThreads) void cv_copy_odd_kernel(const float *Fs, const float *Bs,
                                                                 float *F, float *B, size_t n,
                                                                 const int *count) {
    if ((count[0] & 1) == 0) return;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < 3 * n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        F[p] = Fs[p];
        B[p] = Bs[p];
    }
}

__global__ void cv_begin_kernel(int *stop, int *count) {
    if (threadIdx.x == 0) {
        stop[0] = 0;
        count[0] = 0;
    }
}

// Fused passes (two sweeps per memory round trip) run on the LDS tile kernel up to tile_max_px
// and on the streaming kernel above, except where a level's float32 state (6 planes, one buffer
// resource) would reach 4 GiB, the reach of the streaming kernel's addressing.
long cp_tile_max(const fge_params &p) {
    return p.tile_max_px == 0 ? kTileMaxPxDefault : (p.tile_max_px < 0 ? 0 : p.tile_max_px);
}
bool cp_use_tile(long px, const fge_params &p) {
    return px <= cp_tile_max(p) || 24LL * px >= (1LL << 32);
}

template <typename T>
__global__ __launch_bounds__(kCvThreads) void cp_to_f32_kernel(const T *I, const T *A, float *out,
                                                               size_t n) {
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < 4 * n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads)
        out[p] = static_cast<float>(p < 3 * n ? I[p] : A[p - 3 * n]);
}

// Workspace: the naive plan's ping-pong level buffers (storage type), the float32 working state
// and the float32 Jacobi temporary (6 planes at full size each), the energy partial sums, and a
// small block of scalars.
struct CvLayout {
    size_t work = 0, temp = 0, lvin = 0, rows = 0, in32 = 0, part = 0, scal = 0, total = 0;
};

size_t a256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

CvLayout cv_layout(const Plan &pl, bool jacobi, bool smooth) {
    CvLayout L;
    size_t off = a256(pl.ws_bytes);
    const size_t planes6 = a256(6 * static_cast<size_t>(pl.W) * pl.H * sizeof(float));
    L.work = off;
    off += planes6;
    // the smooth red-black variant sweeps on the fused kernels (cv_fused_sweeps): a second state
    // buffer, and float32 copies of binary16 full-resolution inputs (4 planes)
    const bool fused = smooth && !jacobi;
    L.temp = off;
    off += jacobi || fused ? planes6 : 0;
    L.in32 = off;
    off += fused && pl.elem == 2 ? a256(4 * static_cast<size_t>(pl.W) * pl.H * sizeof(float)) : 0;
    // smooth variant: the area-resized I and alpha of a level below full size (4 float planes)
    // and the row pass of that resize (4 planes of w x H), at the largest such level
    size_t lv_px = 0, rows_px = 0;
    for (int j = 0; smooth && j < pl.n; ++j) {
        if (pl.lv[j].w == pl.W && pl.lv[j].h == pl.H) continue;
        lv_px = std::max(lv_px, static_cast<size_t>(pl.lv[j].w) * pl.lv[j].h);
        rows_px = std::max(rows_px, static_cast<size_t>(pl.lv[j].w) * pl.H);
    }
    L.lvin = off;
    off += a256(4 * lv_px * sizeof(float));
    L.rows = off;
    off += a256(4 * rows_px * sizeof(float));
    L.part = off;
    off += a256(static_cast<size_t>(energy_blocks(pl.W, pl.H)) * 5 * sizeof(double));
    L.scal = off;
    off += 256 + a256(kMaxLevels * sizeof(int));
    L.total = off;
    return L;
}

// The plan of the level loop: every level on per-level kernels (no coarse block, no fused levels).
fge_status cv_plan(int W, int H, const fge_params &p, Plan *pl) {
    fge_params q = p;
    q.kernel = FGE_KERNEL_NAIVE;
    q.coarse_max_px = -1;
    return make_plan(W, H, q, pl);
}

// The sweeps of one level (and, in the convergence form, its energies and stop decisions), with
// I and alpha of type TI read from Wi x Hi through the level's nearest map (the identity for the
// smooth variant's level copies and for a full-size level).
template <typename TI>
fge_status cv_sweep_level(const fge_params &p, const TI *I, const TI *A, int Wi, int Hi, int ti,
                          float *Fo, float *Bo, float *Ft, float *Bt, int w, int h, bool conv,
                          double tol, int kmax, int *stop, int *count, double *part, double *enow,
                          double *eprev, hipStream_t s) {
    const size_t n = static_cast<size_t>(w) * h;
    const bool jac = p.order == FGE_JACOBI;
    const int *guard = conv ? stop : nullptr;
    if (conv) {
        hipLaunchKernelGGL(cv_begin_kernel, dim3(1), dim3(64), 0, s, stop, count);
        if (launch_energy_check(I, A, Wi, Hi, Fo, Bo, w, h, p.omega, p.eps_r, ti, FGE_F32, part,
                                enow, eprev, stop, count, tol, 0, kmax, s))
            return FGE_EHIP;
    }
    for (int k = 1; k <= kmax; ++k) {
        // Jacobi: sweep k reads one buffer and writes the other (odd k: Fo -> Ft)
        float *Fd = jac && (k & 1) ? Ft : Fo, *Bd = jac && (k & 1) ? Bt : Bo;
        if (jac) {
            const float *Fs = (k & 1) ? Fo : Ft, *Bs = (k & 1) ? Bo : Bt;
            hipLaunchKernelGGL(cv_jacobi_kernel<TI>, dim3(blocks_for(n)), dim3(kCvThreads), 0, s, I,
                               A, Wi, Hi, Fs, Bs, Fd, Bd, w, h, p.omega, p.eps_r, guard);
        } else {
            const size_t npairs = static_cast<size_t>((w + 1) >> 1) * h;
            for (int colour = 0; colour < 2; ++colour)
                hipLaunchKernelGGL(cv_halfsweep_kernel<TI>, dim3(blocks_for(npairs)),
                                   dim3(kCvThreads), 0, s, I, A, Wi, Hi, Fo, Bo, w, h, colour,
                                   p.omega, p.eps_r, guard);
        }
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
        if (conv &&
            launch_energy_check(I, A, Wi, Hi, Fd, Bd, w, h, p.omega, p.eps_r, ti, FGE_F32, part,
                                enow, eprev, stop, count, tol, k, kmax, s))
            return FGE_EHIP;
    }
    if (jac && conv) {   // the sweeps that ran decide where the result is
        hipLaunchKernelGGL(cv_copy_odd_kernel, dim3(blocks_for(3 * n)), dim3(kCvThreads), 0, s, Ft,
                           Bt, Fo, Bo, n, count);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
    } else if (jac && (kmax & 1)) {
        hipLaunchKernelGGL(cv_copy_kernel<float>, dim3(blocks_for(3 * n)), dim3(kCvThreads), 0, s,
                           Ft, Bt, Fo, Bo, n, nullptr);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
    }
    return FGE_OK;
}

// The fixed sweep count kmax of a smooth red-black level on the fused kernels: kmax / 2 passes
// of two sweeps, each from one float32 state buffer of the level's size into the other (so the
// previous state is read through the identity map), then one sweep on the per-level kernels when
// kmax is odd.  I and alpha: float32 planes of Wi x Hi (the level's area copy, or full
// resolution).  *out receives the buffer that holds the result (F, then B three planes on).
fge_status cv_fused_sweeps(const fge_params &p, const float *I, const float *A, int Wi, int Hi,
                           float *S0, float *S1, int w, int h, int kmax, float **out, hipStream_t s) {
    const size_t n = static_cast<size_t>(w) * h;
    const bool tile = cp_use_tile(static_cast<long>(n), p);
    float *src = S0, *dst = S1;
    for (int k = 0; k + 2 <= kmax; k += 2) {
        LevelIO io{};
        io.I = I;
        io.A = A;
        io.W = Wi;
        io.H = Hi;
        io.Fp = src;
        io.Bp = src + 3 * n;
        io.wp = w;
        io.hp = h;
        io.Fo = dst;
        io.Bo = dst + 3 * n;
        io.w = w;
        io.h = h;
        io.omega = p.omega;
        io.eps = p.eps_r;
        if (tile ? launch_fine_tile(io, FGE_F32, s) : launch_fine_fused(io, p.strip_rows, FGE_F32, s))
            return FGE_EHIP;
        std::swap(src, dst);
    }
    *out = src;
    if (kmax & 1)
        return cv_sweep_level<float>(p, I, A, Wi, Hi, FGE_F32, src, src + 3 * n, dst, dst + 3 * n, w,
                                     h, false, 0.0, 1, nullptr, nullptr, nullptr, nullptr, nullptr, s);
    return FGE_OK;
}

template <typename T>
fge_status cv_run(const Plan &pl, const fge_params &p, const void *Iv, const void *Av, void *Fv,
                  void *Bv, int resize, double tol, int max_sweeps, int32_t *sweeps_out, char *ws,
                  hipStream_t s) {
    const bool conv = tol >= 0.0;
    const bool smooth = resize == FGE_RESIZE_SMOOTH;
    const CvLayout L = cv_layout(pl, p.order == FGE_JACOBI, smooth);
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *enow = reinterpret_cast<double *>(ws + L.scal);          // 6 doubles
    double *eprev = enow + 6;
    int *stop = reinterpret_cast<int *>(ws + L.scal + 64);
    int *counts = sweeps_out ? sweeps_out : reinterpret_cast<int *>(ws + L.scal + 256);
    const T *I = static_cast<const T *>(Iv);
    const T *A = static_cast<const T *>(Av);
    // the smooth red-black variant with fixed counts sweeps on the fused kernels
    const bool fused = smooth && !conv && p.order == FGE_REDBLACK && p.kernel != FGE_KERNEL_NAIVE;
    const float *I32 = static_cast<const float *>(Iv), *A32 = static_cast<const float *>(Av);
    if (fused && p.storage == FGE_F16) {
        const size_t N = static_cast<size_t>(pl.W) * pl.H;
        float *in = reinterpret_cast<float *>(ws + L.in32);
        hipLaunchKernelGGL(cp_to_f32_kernel<T>, dim3(blocks_for(4 * N)), dim3(kCvThreads), 0, s, I, A,
                           in, N);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
        I32 = in;
        A32 = in + 3 * N;
    }
    for (int j = 0; j < pl.n; ++j) {
        const LevelIO io = level_io(pl, ws, j, Iv, Av, Fv, Bv, p.omega, p.eps_r);
        const int w = io.w, h = io.h;
        const size_t n = static_cast<size_t>(w) * h;
        float *Fo = reinterpret_cast<float *>(ws + L.work);   // working state of the level
        float *Bo = Fo + 3 * n;
        float *Ft = reinterpret_cast<float *>(ws + L.temp);
        float *Bt = Ft + 3 * n;
        if (smooth)
            hipLaunchKernelGGL(cv_bilinear_kernel<T>, dim3(blocks_for(n)), dim3(kCvThreads), 0, s,
                               static_cast<const T *>(io.Fp), static_cast<const T *>(io.Bp), io.wp,
                               io.hp, Fo, Bo, w, h);
        else
            hipLaunchKernelGGL(cv_upsample_kernel<T>, dim3(blocks_for(n)), dim3(kCvThreads), 0, s,
                               static_cast<const T *>(io.Fp), static_cast<const T *>(io.Bp), io.wp,
                               io.hp, Fo, Bo, w, h);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
        const int kmax = conv ? max_sweeps : pl.lv[j].iters;
        fge_status st;
        float *res = Fo;   // the level's result (F, then B)
        if (smooth && (w != pl.W || h != pl.H)) {
            float *lv = reinterpret_cast<float *>(ws + L.lvin);   // I (3 planes), alpha: w x h
            float *rows = reinterpret_cast<float *>(ws + L.rows);
            const int lgr = area_group_log2(pl.W, w), lgc = area_group_log2(pl.H, h);
            const unsigned bx_r = static_cast<unsigned>(((static_cast<size_t>(w) << lgr) + kCvThreads - 1) / kCvThreads);
            const unsigned bx_c = static_cast<unsigned>(((static_cast<size_t>(w) << lgc) + kCvThreads - 1) / kCvThreads);
            hipLaunchKernelGGL((cv_area_kernel<T, true>), dim3(bx_r, pl.H, 4), dim3(kCvThreads), 0, s,
                               I, A, pl.W, pl.H, w, h, lgr, static_cast<double>(pl.W) / w, rows);
            hipLaunchKernelGGL((cv_area_kernel<float, false>), dim3(bx_c, h, 4), dim3(kCvThreads), 0,
                               s, rows, static_cast<const float *>(nullptr), pl.W, pl.H, w, h, lgc,
                               static_cast<double>(pl.H) / h, lv);
            if (hipGetLastError() != hipSuccess) return FGE_EHIP;
            if (fused)
                st = cv_fused_sweeps(p, lv, lv + 3 * n, w, h, Fo, Ft, w, h, kmax, &res, s);
            else
                st = cv_sweep_level<float>(p, lv, lv + 3 * n, w, h, FGE_F32, Fo, Bo, Ft, Bt, w, h,
                                           conv, tol, kmax, stop, counts + j, part, enow, eprev, s);
        } else if (fused) {
            st = cv_fused_sweeps(p, I32, A32, pl.W, pl.H, Fo, Ft, w, h, kmax, &res, s);
        } else {
            st = cv_sweep_level<T>(p, I, A, pl.W, pl.H, p.storage, Fo, Bo, Ft, Bt, w, h, conv, tol,
                                   kmax, stop, counts + j, part, enow, eprev, s);
        }
        if (st != FGE_OK) return st;
        // the level's state, in the storage type
        hipLaunchKernelGGL(cv_copy_kernel<T>, dim3(blocks_for(3 * n)), dim3(kCvThreads), 0, s, res,
                           res + 3 * n, static_cast<T *>(io.Fo), static_cast<T *>(io.Bo), n, nullptr);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
    }
    return FGE_OK;
}

// ---- the convergence form in passes of two sweeps on the fused kernels -------------------------
//
// Every level runs passes of two red-black sweeps on the fused kernels (the LDS tile kernel for
// levels up to tile_max_px, the streaming kernel above; one memory round trip per pass), the
// first pass resizing from the previous level.  Each pass also reduces the energy of the state it
// starts from (pass k: the energy after pass k - 1; pass 1: the previous level's result as the
// resize leaves it) and writes it to pinned host memory, so the energy after pass k arrives with
// pass k + 1; the host stops the level when a pass changes the energy by at most tol times its
// value before the pass, or after max_passes passes.  The device applies the same rule to the
// same values as it totals each energy, so once a level stops at pass k (reported by pass
// k + 1's total) every later pass of the level returns at once and writes nothing; the passes
// write a ring of output buffers in turn, and with two or more of them pass k + 1 never writes
// pass k's.  So the host can keep passes in flight beyond the one it judges at no risk to the
// accepted state -- kCpDepthSmall on levels of at most kCpSmallPx pixels, whose passes are
// shorter than a host round trip, kCpDepthBig on larger ones (deeper queues only add launches
// beyond the stop).  The leading
// levels that fit the coarse block's LDS (at most coarse_max_px pixels, all that fit when it is
// 0, none when it is -1) run in one launch of the coarse block, which takes the same decisions
// on the device (energy reduced in float64 in the workgroup) with no host round trip.  The state
// stays float32 from level to level (inputs in float16 storage are converted once) and is
// converted to the storage type when the last level is done.

constexpr long kCpSmallPx = 1L << 16;
constexpr int kCpSmallBufs = 3;   // small levels: the accepted state and a ring of 2 outputs
constexpr int kCpBigBufs = 3;     // full-size: likewise
constexpr int kCpDepthSmall = 2;  // passes in flight beyond the one judged
constexpr int kCpDepthBig = 1;
constexpr int kCpSlots = 16;      // energy slots in pinned memory (> passes in flight)
constexpr int kCpSlotDoubles = 8; // a slot: fge_energy's 6 outputs, the pass's number, padding

struct CpLayout {
    size_t big[kCpBigBufs] = {}, small[kCpSmallBufs] = {}, in = 0, lin = 0, rows = 0, zero = 0,
           ctl = 0, part = 0, total = 0;
    int nparts = 0;               // partial sums of the largest pass
};

CpLayout cp_layout(int W, int H, const fge_params &p, bool smooth) {
    CpLayout L;
    const size_t n = static_cast<size_t>(W) * H;
    size_t off = 0;
    for (int k = 0; k < kCpBigBufs; ++k) {
        L.big[k] = off;
        off += a256(6 * n * sizeof(float));
    }
    const size_t ns = std::min<size_t>(n, kCpSmallPx);
    for (int k = 0; k < kCpSmallBufs; ++k) {
        L.small[k] = off;
        off += a256(6 * ns * sizeof(float));
    }
    L.in = off;
    off += p.storage == FGE_F16 ? a256(4 * n * sizeof(float)) : 0;
    // a level's inputs resized once (I, alpha planes), for the levels below full resolution
    const int nl0 = num_levels(W, H);
    size_t lin_px = 0;
    for (int j = 0; j + 1 < nl0; ++j)
        lin_px = std::max(lin_px, static_cast<size_t>(level_size(W, j + 1, nl0)) * level_size(H, j + 1, nl0));
    L.lin = off;
    off += a256(4 * lin_px * sizeof(float));
    // the smooth variant's area resize: its row pass (4 planes of w x H) at the widest level
    size_t rows_px = 0;
    for (int j = 0; smooth && j + 1 < nl0; ++j)
        rows_px = std::max(rows_px, static_cast<size_t>(level_size(W, j + 1, nl0)) * H);
    L.rows = off;
    off += a256(4 * rows_px * sizeof(float));
    L.zero = off;   // the 1 x 1 zero start (6 floats)
    off += 256;
    L.ctl = off;    // the device's copy of the stop rule (PassCtl)
    off += 256;
    const int nl = num_levels(W, H);
    for (int j = 0; j < nl; ++j) {
        LevelIO io{};
        io.W = W;
        io.H = H;
        io.w = io.wp = level_size(W, j + 1, nl);
        io.h = io.hp = level_size(H, j + 1, nl);
        const bool tile = p.order == FGE_JACOBI || cp_use_tile(static_cast<long>(io.w) * io.h, p);
        L.nparts = std::max(L.nparts, pass_energy_parts(io, p.strip_rows, tile));
    }
    L.part = off;
    off += a256(static_cast<size_t>(L.nparts) * 5 * sizeof(double));
    L.total = off;
    return L;
}

// I and alpha of a w x h level from the full-resolution float32 inputs by the nearest map (the
// passes' own map, integer division), into 4 compact planes: every pass of the level then reads
// its inputs with the identity map.
__global__ __launch_bounds__(kCvThreads) void cp_compact_kernel(const float *I, const float *A, int W,
                                                               int H, int w, int h, float *out) {
    const size_t n = static_cast<size_t>(w) * h, N = static_cast<size_t>(W) * H;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kCvThreads + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kCvThreads) {
        const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<size_t>(y) * w);
        const size_t q = static_cast<size_t>(static_cast<long long>(y) * H / h) * W +
                         static_cast<size_t>(static_cast<long long>(x) * W / w);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c * n + p] = I[c * N + q];
        out[3 * n + p] = A[q];
    }
}

__global__ void cp_zero_kernel(float *z) {
    if (threadIdx.x < 6) z[threadIdx.x] = 0.0f;
}

template <typename T>
fge_status cp_run(const void *Iv, const void *Av, int W, int H, const fge_params &p, bool smooth,
                  double tol, int max_passes, void *F, void *B, int32_t *passes_out, char *ws,
                  hipStream_t s) {
    const CpLayout L = cp_layout(W, H, p, smooth);
    const size_t N = static_cast<size_t>(W) * H;
    const float *If = static_cast<const float *>(Iv), *Af = static_cast<const float *>(Av);
    if (p.storage == FGE_F16) {
        float *in = reinterpret_cast<float *>(ws + L.in);
        hipLaunchKernelGGL(cp_to_f32_kernel<T>, dim3(blocks_for(4 * N)), dim3(kCvThreads), 0, s,
                           static_cast<const T *>(Iv), static_cast<const T *>(Av), in, N);
        If = in;
        Af = in + 3 * N;
    }
    float *zero = reinterpret_cast<float *>(ws + L.zero);
    hipLaunchKernelGGL(cp_zero_kernel, dim3(1), dim3(64), 0, s, zero);
    if (hipGetLastError() != hipSuccess) return FGE_EHIP;
    double *part = reinterpret_cast<double *>(ws + L.part);
    PassCtl *ctl = reinterpret_cast<PassCtl *>(ws + L.ctl);

    // pinned, mapped: the energy of the state after pass m of a level (written with pass m + 1)
    // goes to slot m % kCpSlots as fge_energy's 6 outputs, then the pass's sequence number (its
    // index among all passes of the call, from 1), written last: the host polls for that number
    // instead of recording and waiting on an event per pass (after the slots: the pass counts of
    // the coarse block's levels)
    double *host = nullptr, *hdev = nullptr;
    const size_t slot_bytes = kCpSlots * kCpSlotDoubles * sizeof(double);
    if (hipHostMalloc(reinterpret_cast<void **>(&host), slot_bytes + kMaxLevels * sizeof(int),
                      hipHostMallocMapped) != hipSuccess)
        return FGE_ENOMEM;
    fge_status ret = FGE_OK;
    for (int k = 0; k < kCpSlots; ++k) host[k * kCpSlotDoubles + 6] = -1.0;
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&hdev), host, 0) != hipSuccess) ret = FGE_EHIP;

    long base = 0;   // passes of the call before the current level's
    // The energy after pass m of the current level: poll its slot for pass m + 1's number; every
    // 1024 polls ask the stream, which fails on an error, and finding it drained with no number
    // is an error too.
    auto wait = [&](int m) {
        if (ret != FGE_OK) return 0.0;
        volatile double *slot = host + kCpSlotDoubles * (m % kCpSlots);
        const double want = static_cast<double>(base + m + 1);
        for (long it = 1; slot[6] != want; ++it) {
            if ((it & 1023) == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q != hipSuccess && q != hipErrorNotReady) {
                    ret = FGE_EHIP;
                    return 0.0;
                }
                if (q == hipSuccess && slot[6] != want) {
                    ret = FGE_EHIP;
                    return 0.0;
                }
            }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        return static_cast<double>(slot[0]);
    };

    // buffers: ids 0 .. kCpBigBufs - 1 the full-size ring, then the small ring
    auto buf = [&](int id) {
        return reinterpret_cast<float *>(ws + (id < kCpBigBufs ? L.big[id] : L.small[id - kCpBigBufs]));
    };
    const int n = num_levels(W, H);
    int prev = -1, wp = 1, hp = 1;   // the accepted state: buffer id (-1: the zero start), size

    // the coarse block (red-black, nearest resize): the longest prefix of levels that fit its LDS
    // and the limit
    const bool jac = p.order == FGE_JACOBI;
    const int climit = p.coarse_max_px < 0 || smooth || jac
                           ? 0 : (p.coarse_max_px == 0 ? kCoarseMaxPx : p.coarse_max_px);
    int nc = 0;
    while (nc < n) {
        const int w = level_size(W, nc + 1, n), h = level_size(H, nc + 1, n);
        const long px = static_cast<long>(w) * h;
        if (px > climit || px > kCoarseMaxPx || static_cast<long>((w + 1) / 2) * h > kCoarseMaxPairs) break;
        ++nc;
    }
    int *hcounts = reinterpret_cast<int *>(reinterpret_cast<char *>(host) + slot_bytes);
    if (nc > 0 && ret == FGE_OK) {
        CoarseArgs c{};
        for (int l = 0; l < nc; ++l) {
            c.src.I[l] = If;
            c.src.A[l] = Af;
            c.src.W[l] = W;
            c.src.H[l] = H;
            c.lw[l] = level_size(W, l + 1, n);
            c.lh[l] = level_size(H, l + 1, n);
            c.lit[l] = 2;
        }
        c.nc = nc;
        float *dst = buf(kCpBigBufs);
        c.Fo = dst;
        c.Bo = dst + 3 * static_cast<size_t>(c.lw[nc - 1]) * c.lh[nc - 1];
        c.omega = p.omega;
        c.eps = p.eps_r;
        int *dcounts = reinterpret_cast<int *>(reinterpret_cast<char *>(hdev) + slot_bytes);
        if (launch_coarse_converge(c, tol, max_passes, dcounts, s)) ret = FGE_EHIP;
        prev = kCpBigBufs;
        wp = c.lw[nc - 1];
        hp = c.lh[nc - 1];
    }
    for (int j = nc; j < n && ret == FGE_OK; ++j) {
        const int w = level_size(W, j + 1, n), h = level_size(H, j + 1, n);
        const long px = static_cast<long>(w) * h;
        const bool small = px <= kCpSmallPx;
        const int lo = small ? kCpBigBufs : 0, hi_id = small ? kCpBigBufs + kCpSmallBufs : kCpBigBufs;
        int outs[kCpSmallBufs], R = 0;
        for (int id = lo; id < hi_id; ++id)
            if (id != prev && R < kCpSmallBufs - 1) outs[R++] = id;
        // Judging pass k needs pass k + 1 (its energy); passes up to k + 1 + depth are in
        // flight (see above: after a stop at k, the passes from k + 2 on write nothing).
        const int depth = small ? kCpDepthSmall : kCpDepthBig;
        const float *Fprev = prev < 0 ? zero : buf(prev);
        const bool tile = jac || cp_use_tile(px, p);   // the Jacobi order: tile kernel only
        int parts = 0;
        // inputs: full resolution for the finest level, else the level's compact copy
        const float *Il = If, *Al = Af;
        int Wl = W, Hl = H;
        if (w != W || h != H) {
            float *lin = reinterpret_cast<float *>(ws + L.lin);
            if (smooth) {   // the level's area averages
                float *rows = reinterpret_cast<float *>(ws + L.rows);
                const int lgr = area_group_log2(W, w), lgc = area_group_log2(H, h);
                const unsigned bx_r = static_cast<unsigned>(((static_cast<size_t>(w) << lgr) + kCvThreads - 1) / kCvThreads);
                const unsigned bx_c = static_cast<unsigned>(((static_cast<size_t>(w) << lgc) + kCvThreads - 1) / kCvThreads);
                hipLaunchKernelGGL((cv_area_kernel<float, true>), dim3(bx_r, H, 4), dim3(kCvThreads),
                                   0, s, If, Af, W, H, w, h, lgr, static_cast<double>(W) / w, rows);
                hipLaunchKernelGGL((cv_area_kernel<float, false>), dim3(bx_c, h, 4), dim3(kCvThreads),
                                   0, s, rows, static_cast<const float *>(nullptr), W, H, w, h, lgc,
                                   static_cast<double>(H) / h, lin);
            } else {
                hipLaunchKernelGGL(cp_compact_kernel, dim3(blocks_for(static_cast<size_t>(w) * h)),
                                   dim3(kCvThreads), 0, s, If, Af, W, H, w, h, lin);
            }
            if (hipGetLastError() != hipSuccess) ret = FGE_EHIP;
            Il = lin;
            Al = lin + 3 * static_cast<size_t>(w) * h;
            Wl = w;
            Hl = h;
        }
        // The smooth variant's first pass starts from the previous level resized bilinearly to
        // this level's size, put in outs[1] (pass 2 is the first to write it, after pass 1 has
        // read it).
        if (smooth && ret == FGE_OK) {
            float *st = buf(outs[1]);
            const size_t n = static_cast<size_t>(w) * h;
            hipLaunchKernelGGL(cv_bilinear_kernel<float>, dim3(blocks_for(n)), dim3(kCvThreads), 0, s,
                               Fprev, Fprev + 3 * static_cast<size_t>(wp) * hp, wp, hp, st, st + 3 * n,
                               w, h);
            if (hipGetLastError() != hipSuccess) ret = FGE_EHIP;
        }
        // pass k (1-based): from the accepted previous level (smooth: its resize) or from pass
        // k - 1, into outs[(k - 1) % R]; with it, the energy of its start state into slot k - 1
        auto pass = [&](int k) {
            LevelIO io{};
            io.I = Il;
            io.A = Al;
            io.W = Wl;
            io.H = Hl;
            const bool from_prev = k == 1 && !smooth;
            const float *src = from_prev ? Fprev : buf(outs[(k - 2 + R) % R]);
            io.Fp = src;
            io.wp = from_prev ? wp : w;
            io.hp = from_prev ? hp : h;
            io.Bp = src + 3 * static_cast<size_t>(io.wp) * io.hp;
            float *dst = buf(outs[(k - 1) % R]);
            io.Fo = dst;
            io.Bo = dst + 3 * static_cast<size_t>(w) * h;
            io.w = w;
            io.h = h;
            io.omega = p.omega;
            io.eps = p.eps_r;
            if (parts == 0) parts = pass_energy_parts(io, p.strip_rows, tile);
            const int sl = (k - 1) % kCpSlots;
            // the device applies the stop rule too: passes after the one that reports the stop
            // (pass k + 1 reports the energy after pass k) return at once
            if (launch_pass_energy(io, p.strip_rows, tile, part, k == 1 ? nullptr : &ctl->stop, s,
                                   jac) ||
                launch_pass_final(part, parts, hdev + kCpSlotDoubles * sl, ctl, k, tol, base + k, s))
                ret = FGE_EHIP;
        };
        int hi = 0;   // passes enqueued
        auto fill = [&](int upto) {
            while (ret == FGE_OK && hi < std::min(upto, max_passes)) pass(++hi);
        };
        fill(2 + depth);
        double e_prev = wait(0);
        int k = 1;
        for (;;) {
            if (ret != FGE_OK || k >= max_passes) break;
            fill(k + 1 + depth);
            const double e = wait(k);
            if (ret != FGE_OK || std::fabs(e_prev - e) <= tol * e_prev) break;
            e_prev = e;
            ++k;
        }
        if (passes_out) passes_out[j] = k;
        base += hi;
        prev = outs[(k - 1) % R];
        wp = w;
        hp = h;
    }
    if (ret == FGE_OK) {
        const float *Fs = buf(prev);
        hipLaunchKernelGGL(cv_copy_kernel<T>, dim3(blocks_for(3 * N)), dim3(kCvThreads), 0, s, Fs,
                           Fs + 3 * N, static_cast<T *>(F), static_cast<T *>(B), N, nullptr);
        if (hipGetLastError() != hipSuccess) ret = FGE_EHIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess && ret == FGE_OK) ret = FGE_EHIP;
    if (ret == FGE_OK && passes_out)
        for (int l = 0; l < nc; ++l) passes_out[l] = reinterpret_cast<volatile int *>(hcounts)[l];
    (void)hipHostFree(host);
    return ret;
}

}  // namespace

size_t levels_workspace_bytes(int W, int H, const fge_params &p, int resize, int passes) {
    if (passes)
        return converge_passes_workspace_bytes(W, H, p, resize == FGE_RESIZE_SMOOTH);
    Plan pl;
    if (cv_plan(W, H, p, &pl) != FGE_OK) return 0;
    return cv_layout(pl, p.order == FGE_JACOBI, resize == FGE_RESIZE_SMOOTH).total;
}

size_t converge_workspace_bytes(int W, int H, const fge_params &p) {
    return levels_workspace_bytes(W, H, p, FGE_RESIZE_NEAREST, 0);
}

fge_status estimate_levels(const void *I, const void *A, int W, int H, const fge_params &p,
                           int resize, double tol, int max_sweeps, int passes, void *F, void *B,
                           int32_t *sweeps_out, void *workspace, size_t workspace_bytes,
                           void *stream) {
    if (passes != 0 && passes != 1) return FGE_EINVAL;
    if (resize != FGE_RESIZE_NEAREST && resize != FGE_RESIZE_SMOOTH) return FGE_EINVAL;
    if (passes) {   // the test after every pass of two sweeps, on the fused kernels
        // (the pass counts come back to the host, which takes the stop decisions; sweeps_out is
        // device memory here, as in the per-level form)
        int32_t counts[kMaxLevels] = {};
        const fge_status st = estimate_converge_passes(I, A, W, H, p, tol, max_sweeps, F, B, counts,
                                                       workspace, workspace_bytes, stream,
                                                       resize == FGE_RESIZE_SMOOTH);
        if (st != FGE_OK || !sweeps_out) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (hipMemcpyAsync(sweeps_out, counts, num_levels(W, H) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return FGE_EHIP;
        return FGE_OK;
    }
    Plan pl;
    const fge_status st = cv_plan(W, H, p, &pl);
    if (st != FGE_OK) return st;
    if (!I || !A || !F || !B) return FGE_EINVAL;
    if (outputs_alias(I, A, F, B, W, H, p.storage == FGE_F16 ? 2 : 4, workspace, workspace_bytes))
        return FGE_EINVAL;
    if (resize != FGE_RESIZE_NEAREST && resize != FGE_RESIZE_SMOOTH) return FGE_EINVAL;
    if (tol >= 0.0 && (max_sweeps < 1 || max_sweeps > kCvMaxSweeps)) return FGE_EINVAL;
    if (!(tol == tol)) return FGE_EINVAL;   // NaN
    const size_t need = cv_layout(pl, p.order == FGE_JACOBI, resize == FGE_RESIZE_SMOOTH).total;
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return FGE_EWORKSPACE;
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p.storage == FGE_F16)
        return cv_run<_Float16>(pl, p, I, A, F, B, resize, tol, max_sweeps, sweeps_out, ws, s);
    return cv_run<float>(pl, p, I, A, F, B, resize, tol, max_sweeps, sweeps_out, ws, s);
}

fge_status estimate_converge(const void *I, const void *A, int W, int H, const fge_params &p,
                             double tol, int max_sweeps, void *F, void *B, int32_t *sweeps_out,
                             void *workspace, size_t workspace_bytes, void *stream) {
    return estimate_levels(I, A, W, H, p, FGE_RESIZE_NEAREST, tol, max_sweeps, 0, F, B, sweeps_out,
                           workspace, workspace_bytes, stream);
}

size_t converge_passes_workspace_bytes(int W, int H, const fge_params &p, bool smooth) {
    if (W < 1 || H < 1 || W > kMaxSide || H > kMaxSide) return 0;
    return cp_layout(W, H, p, smooth).total;
}

fge_status estimate_converge_passes(const void *I, const void *A, int W, int H,
                                    const fge_params &p, double tol, int max_passes, void *F,
                                    void *B, int32_t *passes_out, void *workspace,
                                    size_t workspace_bytes, void *stream, bool smooth) {
    if (!params_valid(p)) return FGE_EINVAL;
    if (W < 1 || H < 1 || W > kMaxSide || H > kMaxSide) return FGE_EINVAL;
    if (!I || !A || !F || !B) return FGE_EINVAL;
    if (!(tol >= 0.0) || !std::isfinite(tol) || max_passes < 1 || max_passes > kCvMaxSweeps)
        return FGE_EINVAL;
    if (outputs_alias(I, A, F, B, W, H, p.storage == FGE_F16 ? 2 : 4, workspace, workspace_bytes))
        return FGE_EINVAL;
    const size_t need = converge_passes_workspace_bytes(W, H, p, smooth);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return FGE_EWORKSPACE;
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p.storage == FGE_F16)
        return cp_run<_Float16>(I, A, W, H, p, smooth, tol, max_passes, F, B, passes_out, ws, s);
    return cp_run<float>(I, A, W, H, p, smooth, tol, max_passes, F, B, passes_out, ws, s);
}

}  // namespace fge

extern "C" {

size_t fge_converge_passes_workspace_bytes(int32_t H, int32_t W, const fge_params *p) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    return fge::converge_passes_workspace_bytes(W, H, *p);
}

fge_status fge_estimate_foreground_converge_passes(const void *I, const void *alpha, int32_t H,
                                                   int32_t W, const fge_params *p, double tol,
                                                   int32_t max_passes, void *F, void *B,
                                                   int32_t *passes_out, void *workspace,
                                                   size_t workspace_bytes, void *stream) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    return fge::estimate_converge_passes(I, alpha, W, H, *p, tol, max_passes, F, B, passes_out,
                                         workspace, workspace_bytes, stream);
}


size_t fge_converge_workspace_bytes(int32_t H, int32_t W, const fge_params *p) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    return fge::converge_workspace_bytes(W, H, *p);
}

size_t fge_levels_workspace_bytes(int32_t H, int32_t W, const fge_params *p,
                                  const fge_level_options *o) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    if (!o || o->size != sizeof(fge_level_options)) return 0;
    return fge::levels_workspace_bytes(W, H, *p, o->resize, o->passes);
}

fge_status fge_estimate_foreground_levels(const void *I, const void *alpha, int32_t H, int32_t W,
                                          const fge_params *p, const fge_level_options *o,
                                          void *F, void *B, int32_t *sweeps_out, void *workspace,
                                          size_t workspace_bytes, void *stream) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    if (!o || o->size != sizeof(fge_level_options)) return FGE_EINVAL;
    return fge::estimate_levels(I, alpha, W, H, *p, o->resize, o->tol, o->max_sweeps, o->passes, F,
                                B, sweeps_out, workspace, workspace_bytes, stream);
}

fge_status fge_estimate_foreground_converge(const void *I, const void *alpha, int32_t H, int32_t W,
                                            const fge_params *p, double tol, int32_t max_sweeps,
                                            void *F, void *B, int32_t *sweeps_out, void *workspace,
                                            size_t workspace_bytes, void *stream) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    return fge::estimate_converge(I, alpha, W, H, *p, tol, max_sweeps, F, B, sweeps_out, workspace,
                                  workspace_bytes, stream);
}

}  // extern "C"
