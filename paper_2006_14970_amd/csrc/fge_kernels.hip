// HIP kernels (gfx950) for multi-level foreground estimation, arXiv 2006.14970, Algorithm 1.
//
// Three kernel families, all computing in float32 and storing in T (float or _Float16):
//
//  coarse_kernel   One workgroup runs every level whose w*h <= 4096 entirely in LDS (alpha, F
//                  and B planes, 112 KB), including the 10-sweep low-resolution levels, then
//                  writes the last of those levels to memory.  Removes ~100 dependent launches.
//
//  fine_kernel     One launch per fine level.  Each wave owns a strip of 128 columns (a pair of
//                  adjacent pixels per lane, so every lane has exactly one pixel of each colour)
//                  and streams down its rows: for every new row it gathers I and alpha from the
//                  full-resolution input (nearest), upsamples F and B from the previous level,
//                  and runs all four red-black half-sweeps of the level's two sweeps on a
//                  six-row register window (temporal blocking).  Horizontal neighbours cross
//                  lanes with DPP; nothing goes through LDS.  A half-sweep invalidates one ring
//                  at the strip edge, so strips overlap by 4 rows/columns of halo that are
//                  computed but not stored.  One HBM round trip per level.
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

// Reciprocal with v_rcp_f32 (1 ulp); its arguments here are in [0.02, 4].
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Makes a value that is the same in every lane of the wave visible as such to the compiler, so
// that branches on it are scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

__device__ __forceinline__ float weight(float a, float b, float omega, float eps) {
    return fmaf(omega, fabsf(a - b), eps);
}

// ------------------------------------------------------------------------------------------
// Coarse kernel: levels [0, nc) in LDS.
// ------------------------------------------------------------------------------------------

struct CoarseArgs {
    const void *I;
    const void *A;
    int W, H;
    void *Fo;
    void *Bo;
    int nc;
    int lw[kMaxLevels], lh[kMaxLevels], lit[kMaxLevels];
    float omega, eps;
};

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void coarse_kernel(CoarseArgs args) {
    __shared__ float sA[kCoarseMaxPx];
    __shared__ float sF[3 * kCoarseMaxPx];
    __shared__ float sB[3 * kCoarseMaxPx];

    const T *I = static_cast<const T *>(args.I);
    const T *A = static_cast<const T *>(args.A);
    const int W = args.W, H = args.H;
    const size_t planeI = static_cast<size_t>(W) * H;
    const int tid = threadIdx.x;
    const float omega = args.omega, eps = args.eps;

    int wp = 1, hp = 1;
    for (int l = 0; l < args.nc; ++l) {
        const int w = args.lw[l], h = args.lh[l], iters = args.lit[l];
        const int n = w * h;

        // Resize: alpha from the full-resolution matte, F and B from the previous level (the
        // level before the first is the 1x1 zero start).  Gather into registers first, since
        // the new level overwrites the old one in place.
        float ra[kCoarsePxPerThread], rf[kCoarsePxPerThread][3], rb[kCoarsePxPerThread][3];
#pragma unroll
        for (int k = 0; k < kCoarsePxPerThread; ++k) {
            const int p = tid + k * kCoarseThreads;
            ra[k] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) rf[k][c] = rb[k][c] = 0.0f;
            if (p < n) {
                const int y = p / w, x = p - y * w;
                ra[k] = ldf(A + static_cast<size_t>(y * H / h) * W + x * W / w);
                if (l > 0) {
                    const int q = (y * hp / h) * wp + x * wp / w;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        rf[k][c] = sF[c * kCoarseMaxPx + q];
                        rb[k][c] = sB[c * kCoarseMaxPx + q];
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCoarsePxPerThread; ++k) {
            const int p = tid + k * kCoarseThreads;
            if (p < n) {
                sA[p] = ra[k];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sF[c * kCoarseMaxPx + p] = rf[k][c];
                    sB[c * kCoarseMaxPx + p] = rb[k][c];
                }
            }
        }
        __syncthreads();

        // Sweeps: each half-sweep updates one colour; thread q owns the pair of columns
        // (2j, 2j+1) of row y and updates the one of the current colour.
        const int pw = (w + 1) >> 1;
        const int npairs = pw * h;
        for (int it = 0; it < iters; ++it) {
            for (int colour = 0; colour < 2; ++colour) {
                for (int q = tid; q < npairs; q += kCoarseThreads) {
                    const int y = q / pw;
                    const int x = 2 * (q - y * pw) + ((y + colour) & 1);
                    if (x < w) {
                        const int i = y * w + x;
                        const float a = sA[i];
                        const int nb[4] = {y * w + (x > 0 ? x - 1 : 0), y * w + (x < w - 1 ? x + 1 : w - 1),
                                           (y > 0 ? y - 1 : 0) * w + x, (y < h - 1 ? y + 1 : h - 1) * w + x};
                        float s[4], S = 0.0f;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            s[j] = weight(a, sA[nb[j]], omega, eps);
                            S += s[j];
                        }
                        const float iS = 1.0f / S;
                        const float b = 1.0f - a;
                        const float k = 1.0f / (S + fmaf(a, a, b * b));
                        const size_t src = static_cast<size_t>(y * H / h) * W + x * W / w;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float P = 0.0f, Q = 0.0f;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                P = fmaf(s[j], sF[c * kCoarseMaxPx + nb[j]], P);
                                Q = fmaf(s[j], sB[c * kCoarseMaxPx + nb[j]], Q);
                            }
                            const float fb = P * iS, bb = Q * iS;
                            const float r = ldf(I + c * planeI + src) - a * fb - b * bb;
                            sF[c * kCoarseMaxPx + i] = clamp01(fmaf(a * k, r, fb));
                            sB[c * kCoarseMaxPx + i] = clamp01(fmaf(b * k, r, bb));
                        }
                    }
                }
                __syncthreads();
            }
        }
        wp = w;
        hp = h;
    }

    // Write the last coarse level.
    T *Fo = static_cast<T *>(args.Fo);
    T *Bo = static_cast<T *>(args.Bo);
    const int n = wp * hp;
    for (int p = tid; p < n; p += kCoarseThreads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            stf(Fo + static_cast<size_t>(c) * n + p, sF[c * kCoarseMaxPx + p]);
            stf(Bo + static_cast<size_t>(c) * n + p, sB[c * kCoarseMaxPx + p]);
        }
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
constexpr int kWin = kNHS + 2;          // rows held per wave: r-1 .. r+NHS
constexpr int kHalo = kNHS;             // invalid ring after kNHS half-sweeps
constexpr int kStripCols = 128;         // two columns per lane
constexpr int kFirstCore = kStripCols - kHalo;          // strip 0 keeps columns [0, 124)
constexpr int kMidCore = kStripCols - 2 * kHalo;        // interior strips keep 120 columns
constexpr int kPD = 2;                  // rows prefetched ahead
constexpr int kWavesPerBlock = 4;

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

// Number of column strips for a level of width w (see the geometry in fine_kernel).
__host__ __device__ inline int fine_strips_x(int w) {
    if (w <= kStripCols) return 1;
    const int rest = w - (kFirstCore + kFirstCore);
    return 2 + (rest > 0 ? (rest + kMidCore - 1) / kMidCore : 0);
}

template <typename T>
struct Raw {
    T a[2];
    T i[2][3];
    T f[2][3];
    T b[2][3];
};

// Per-wave constants of a strip.  Every image plane has its own base pointer (uniform, kept in
// SGPRs) and is addressed with 32-bit byte offsets: one plane holds at most 32767^2 elements,
// whose float32 byte offsets still fit in 32 bits, so the loads use the scalar-base form.
template <typename T>
struct FineGeo {
    const char *I[3], *A, *Fp[3], *Bp[3];
    char *Fo[3], *Bo[3];
    int W, H, wp, hp, w, h;
    uint32_t sia, sib, spa, spb;   // byte offsets of this lane's source columns
    uint32_t oxa, oxb;             // byte offsets of this lane's output columns
    bool store_a, store_b;         // columns inside this strip's core
    bool edge_a, edge_b;           // column == w - 1 (right border inside the wave)
    int y0, y1, t0, tlast;
    float omega, eps;
};

// Register window: row slot = (row - t0) mod kWin, column of the lane's pair.
struct FineWin {
    float al[kWin][2];
    float iv[kWin][2][3];
    float fv[kWin][2][3];
    float bv[kWin][2][3];
    float wl[kWin][2], wr[kWin][2], wu[kWin][2], wd[kWin][2], ka[kWin][2], kb[kWin][2];
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

template <typename T>
__device__ __forceinline__ T ldb(const char *base, uint32_t off) {
    return *reinterpret_cast<const T *>(base + off);
}

template <typename T>
__device__ __forceinline__ void stb(char *base, uint32_t off, float v) {
    *reinterpret_cast<T *>(base + off) = static_cast<T>(v);
}

// Gather one row: I and alpha from input row qi (nearest), F and B from previous-level row qp.
template <typename T>
__device__ __forceinline__ void fine_load_row(const FineGeo<T> &g, Raw<T> &r, int qi, int qp) {
    const uint32_t ri = static_cast<uint32_t>(qi) * static_cast<uint32_t>(g.W) * sizeof(T);
    const uint32_t rp = static_cast<uint32_t>(qp) * static_cast<uint32_t>(g.wp) * sizeof(T);
    const uint32_t ia = ri + g.sia, ib = ri + g.sib, pa = rp + g.spa, pb = rp + g.spb;
    r.a[0] = ldb<T>(g.A, ia);
    r.a[1] = ldb<T>(g.A, ib);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r.i[0][c] = ldb<T>(g.I[c], ia);
        r.i[1][c] = ldb<T>(g.I[c], ib);
        r.f[0][c] = ldb<T>(g.Fp[c], pa);
        r.f[1][c] = ldb<T>(g.Fp[c], pb);
        r.b[0][c] = ldb<T>(g.Bp[c], pa);
        r.b[1][c] = ldb<T>(g.Bp[c], pb);
    }
}

template <int R, typename T>
__device__ __forceinline__ void fine_consume(FineWin &v, const Raw<T> &r) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        v.al[R][s] = static_cast<float>(r.a[s]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v.iv[R][s][c] = static_cast<float>(r.i[s][c]);
            v.fv[R][s][c] = static_cast<float>(r.f[s][c]);
            v.bv[R][s][c] = static_cast<float>(r.b[s][c]);
        }
    }
}

// Weights of row r (slot R) from its own and its neighbours' alpha (rows in slots U and D).
// Rows -1 and h are phantom rows outside the image: the neighbour clamp of Algorithm 1 makes a
// border pixel its own neighbour, and the phantom row holds exactly that value, because its
// "update" copies the adjacent image row (weights 1 toward it, 0 elsewhere, no data term).
// Rows beyond the phantom rows are loaded from the clamped border row and never feed a stored
// result.
template <int R, int U, int D, bool EDGE, bool BORDER, typename T>
__device__ __forceinline__ void fine_constants(FineWin &v, const FineGeo<T> &g, int r) {
    const float omega = g.omega, eps = g.eps;
    const float a0 = v.al[R][0], a1 = v.al[R][1];
    const float l0 = from_left(v.al[R][1], a0);        // left of column a: lane-1's column b
    float r1 = from_right(v.al[R][0], a1);             // right of column b: lane+1's column a
    float r0 = a1;
    if (EDGE) {
        r0 = g.edge_a ? a0 : r0;
        r1 = g.edge_b ? a1 : r1;
    }
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
template <int R, int U, int D, int S, bool EDGE, typename T>
__device__ __forceinline__ void fine_update(FineWin &v, const FineGeo<T> &g) {
    const float a = v.al[R][S], b = 1.0f - a;
    const float cl = v.wl[R][S], cr = v.wr[R][S], cu = v.wu[R][S], cd = v.wd[R][S];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float fs = v.fv[R][S][c], bs = v.bv[R][S][c];
        float fL, fR, bL, bR;
        if (S == 0) {
            fL = from_left(v.fv[R][1][c], fs);
            bL = from_left(v.bv[R][1][c], bs);
            fR = v.fv[R][1][c];
            bR = v.bv[R][1][c];
            if (EDGE) {
                fR = g.edge_a ? fs : fR;
                bR = g.edge_a ? bs : bR;
            }
        } else {
            fL = v.fv[R][0][c];
            bL = v.bv[R][0][c];
            fR = from_right(v.fv[R][0][c], fs);
            bR = from_right(v.bv[R][0][c], bs);
            if (EDGE) {
                fR = g.edge_b ? fs : fR;
                bR = g.edge_b ? bs : bR;
            }
        }
        const float fb = fmaf(cd, v.fv[D][S][c], fmaf(cu, v.fv[U][S][c], fmaf(cr, fR, cl * fL)));
        const float bb = fmaf(cd, v.bv[D][S][c], fmaf(cu, v.bv[U][S][c], fmaf(cr, bR, cl * bL)));
        const float r = v.iv[R][S][c] - a * fb - b * bb;
        v.fv[R][S][c] = clamp01(fmaf(v.ka[R][S], r, fb));
        v.bv[R][S][c] = clamp01(fmaf(v.kb[R][S], r, bb));
    }
}

template <int R, typename T>
__device__ __forceinline__ void fine_store_row(const FineWin &v, const FineGeo<T> &g, int r) {
    const uint32_t ro = static_cast<uint32_t>(r) * static_cast<uint32_t>(g.w) * sizeof(T);
    const uint32_t oa = ro + g.oxa, ob = ro + g.oxb;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (g.store_a) {
            stb<T>(g.Fo[c], oa, v.fv[R][0][c]);
            stb<T>(g.Bo[c], oa, v.bv[R][0][c]);
        }
        if (g.store_b) {
            stb<T>(g.Fo[c], ob, v.fv[R][1][c]);
            stb<T>(g.Bo[c], ob, v.bv[R][1][c]);
        }
    }
}

// One pipeline step at row t (TT = (t - t0) mod 6): take row t from the prefetch buffer and
// prefetch row t + kPD, compute the weights of row t-1, run half-sweep k on row t-1-k for
// k = 0..3, and store row t-4, which has now seen both sweeps.
template <int TT, bool EDGE, bool BORDER, typename T>
__device__ __forceinline__ void fine_step(FineWin &v, Raw<T> (&raw)[kPD], const FineGeo<T> &g,
                                          RowMap &mi, RowMap &mp, int t) {
    constexpr int S = (TT + 1) & 1;       // column of the pair updated in this step
    fine_consume<TT % kWin>(v, raw[TT % kPD]);
    {
        const int tl = t + kPD;
        if (tl >= 1 && tl <= g.h - 1) {
            mi.advance();
            mp.advance();
        }
        fine_load_row(g, raw[TT % kPD], mi.q, mp.q);
    }
    fine_constants<(TT + 5) % kWin, (TT + 4) % kWin, TT % kWin, EDGE, BORDER>(v, g, t - 1);
    fine_update<(TT + 5) % kWin, (TT + 4) % kWin, TT % kWin, S, EDGE>(v, g);
    fine_update<(TT + 4) % kWin, (TT + 3) % kWin, (TT + 5) % kWin, S, EDGE>(v, g);
    fine_update<(TT + 3) % kWin, (TT + 2) % kWin, (TT + 4) % kWin, S, EDGE>(v, g);
    fine_update<(TT + 2) % kWin, (TT + 1) % kWin, (TT + 3) % kWin, S, EDGE>(v, g);
    if (t - 4 >= g.y0 && t - 4 < g.y1) fine_store_row<(TT + 2) % kWin>(v, g, t - 4);
    // keep the scheduler from interleaving consecutive steps, which only raises register pressure
    __builtin_amdgcn_sched_barrier(0);
}

template <bool EDGE, bool BORDER, typename T>
__device__ __forceinline__ void fine_block(FineWin &v, Raw<T> (&raw)[kPD], const FineGeo<T> &g,
                                           RowMap &mi, RowMap &mp, int t) {
    fine_step<0, EDGE, BORDER>(v, raw, g, mi, mp, t);
    fine_step<1, EDGE, BORDER>(v, raw, g, mi, mp, t + 1);
    fine_step<2, EDGE, BORDER>(v, raw, g, mi, mp, t + 2);
    fine_step<3, EDGE, BORDER>(v, raw, g, mi, mp, t + 3);
    fine_step<4, EDGE, BORDER>(v, raw, g, mi, mp, t + 4);
    fine_step<5, EDGE, BORDER>(v, raw, g, mi, mp, t + 5);
}

template <typename T, bool EDGE>
__device__ __forceinline__ void fine_strip(const FineArgs &args, int sx, int sy, int lane) {
    FineGeo<T> g;
    const size_t planeI = static_cast<size_t>(args.W) * args.H * sizeof(T);
    const size_t planeP = static_cast<size_t>(args.wp) * args.hp * sizeof(T);
    const size_t planeO = static_cast<size_t>(args.w) * args.h * sizeof(T);
    g.A = static_cast<const char *>(args.A);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        g.I[c] = static_cast<const char *>(args.I) + c * planeI;
        g.Fp[c] = static_cast<const char *>(args.Fp) + c * planeP;
        g.Bp[c] = static_cast<const char *>(args.Bp) + c * planeP;
        g.Fo[c] = static_cast<char *>(args.Fo) + c * planeO;
        g.Bo[c] = static_cast<char *>(args.Bo) + c * planeO;
    }
    g.W = args.W;
    g.H = args.H;
    g.wp = args.wp;
    g.hp = args.hp;
    g.w = args.w;
    g.h = args.h;
    g.omega = args.omega;
    g.eps = args.eps;
    const int w = args.w, h = args.h, nx = args.nx;

    // Column geometry.  Strip 0 starts at column 0 (its left edge is the image border, so DPP
    // lane 0 sees itself, which is the clamp); the last strip ends at column w-1 (lane 63 sees
    // itself); interior strips keep 120 core columns.  EDGE: a single strip narrower than 128.
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
    g.edge_a = xa == w - 1;
    g.edge_b = xb == w - 1;

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
#pragma unroll
    for (int r = 0; r < kWin; ++r)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            v.al[r][s] = 0.0f;
            v.wl[r][s] = v.wr[r][s] = v.wu[r][s] = v.wd[r][s] = v.ka[r][s] = v.kb[r][s] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) v.iv[r][s][c] = v.fv[r][s][c] = v.bv[r][s][c] = 0.0f;
        }
    // Row maps for the clamped rows t0, t0+1, ...: input row and previous-level row.
    RowMap mi, mp;
    const int tc0 = min(max(g.t0, 0), h - 1);
    mi.init(tc0, args.H, h);
    mp.init(tc0, args.hp, h);
    Raw<T> raw[kPD];
    fine_load_row(g, raw[0], mi.q, mp.q);
#pragma unroll
    for (int k = 1; k < kPD; ++k) {
        const int tl = g.t0 + k;
        if (tl >= 1 && tl <= h - 1) {
            mi.advance();
            mp.advance();
        }
        fine_load_row(g, raw[k], mi.q, mp.q);
    }

    // Phantom rows -1 and h get their weights at steps 0 and h + 1.  Only the blocks holding
    // those steps use the border variant: the first block of a top strip, and the blocks from
    // the one holding step h + 1 on.  The regions run one after the other (not as alternatives
    // inside one loop), which keeps the register allocation of the steady state spill-free.
    int t = g.t0;
    if (t <= 0) {
        fine_block<EDGE, true>(v, raw, g, mi, mp, t);
        t += kWin;
    }
    for (; t <= g.tlast && t + kWin <= h + 1; t += kWin) fine_block<EDGE, false>(v, raw, g, mi, mp, t);
    for (; t <= g.tlast; t += kWin) fine_block<EDGE, true>(v, raw, g, mi, mp, t);
}

template <typename T>
__global__ __launch_bounds__(64 * kWavesPerBlock, 2) void fine_kernel(FineArgs args) {
    const int wave = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= args.nx * args.ny) return;
    const int lane = threadIdx.x & 63;
    const int sx = wave % args.nx, sy = wave / args.nx;
    if (args.w < kStripCols)
        fine_strip<T, true>(args, sx, sy, lane);
    else
        fine_strip<T, false>(args, sx, sy, lane);
}

template <typename T>
int launch_coarse_t(const Plan &plan, const void *I, const void *A, void *Fo, void *Bo,
                    float omega, float eps, hipStream_t s) {
    CoarseArgs a{};
    a.I = I;
    a.A = A;
    a.W = plan.W;
    a.H = plan.H;
    a.Fo = Fo;
    a.Bo = Bo;
    a.nc = plan.nc;
    for (int i = 0; i < plan.nc; ++i) {
        a.lw[i] = plan.lv[i].w;
        a.lh[i] = plan.lv[i].h;
        a.lit[i] = plan.lv[i].iters;
    }
    a.omega = omega;
    a.eps = eps;
    hipLaunchKernelGGL(coarse_kernel<T>, dim3(1), dim3(kCoarseThreads), 0, s, a);
    return static_cast<int>(hipGetLastError());
}

int auto_strip_rows(int w, int h) {
    // Aim at about one wave per SIMD (256 CUs x 4) and at least 8 core rows per strip.
    const long nx = fine_strips_x(w);
    long rows = (static_cast<long>(h) * nx + 1023) / 1024;
    rows = (rows + 1) & ~1L;
    if (rows < 8) rows = 8;
    if (rows > h) rows = h;
    return static_cast<int>(rows);
}

template <typename T>
int launch_fine_t(const LevelIO &io, int strip_rows, hipStream_t s) {
    FineArgs a{};
    a.I = io.I;
    a.A = io.A;
    a.W = io.W;
    a.H = io.H;
    a.Fp = io.Fp;
    a.Bp = io.Bp;
    a.wp = io.wp;
    a.hp = io.hp;
    a.Fo = io.Fo;
    a.Bo = io.Bo;
    a.w = io.w;
    a.h = io.h;
    a.omega = io.omega;
    a.eps = io.eps;
    a.nx = fine_strips_x(io.w);
    a.strip_rows = strip_rows > 0 ? strip_rows : auto_strip_rows(io.w, io.h);
    a.ny = (io.h + a.strip_rows - 1) / a.strip_rows;
    const int waves = a.nx * a.ny;
    const int blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(fine_kernel<T>, dim3(blocks), dim3(64 * kWavesPerBlock), 0, s, a);
    return static_cast<int>(hipGetLastError());
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

}  // namespace

int launch_coarse(const Plan &plan, const void *I, const void *A, void *Fo, void *Bo,
                  float omega, float eps, int storage, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (storage == FGE_F16) return launch_coarse_t<_Float16>(plan, I, A, Fo, Bo, omega, eps, s);
    return launch_coarse_t<float>(plan, I, A, Fo, Bo, omega, eps, s);
}

int launch_fine_fused(const LevelIO &io, int strip_rows, int storage, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (storage == FGE_F16) return launch_fine_t<_Float16>(io, strip_rows, s);
    return launch_fine_t<float>(io, strip_rows, s);
}

int launch_naive_level(const LevelIO &io, int iters, int storage, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (storage == FGE_F16) return launch_naive_t<_Float16>(io, iters, s);
    return launch_naive_t<float>(io, iters, s);
}

}  // namespace fge
