// Closed-form foreground estimation (Section III-B, eq. 2) as a preconditioned conjugate-gradient
// solve on the device (C ABI in include/fge.h: fge_closed_form).
//
// The cost of eq. 2, per colour channel, with every edge weight raised by the regulariser eps
// (the paper introduces eps_r in Section III-C because F is free where alpha = 0 and B where
// alpha = 1, which leaves eq. 2 alone singular):
//   E(F, B) = sum_i (a_i F_i + (1 - a_i) B_i - I_i)^2
//           + sum over horizontal and vertical neighbour pairs {i, j} of
//             w_ij ((F_i - F_j)^2 + (B_i - B_j)^2),   w_ij = eps + omega |a_i - a_j|,
// eq. 2's |alpha_x| and |alpha_y| read as forward differences (omega = 1 is eq. 2 as printed).
// Its minimiser solves the 2n x 2n system A x = b, with x_i = (F_i, B_i) and U_i = (a_i, 1 - a_i):
//   (A x)_i = U_i (U_i . x_i) + sum_j w_ij (x_i - x_j),   b_i = U_i I_i.
// The same A serves the three channels; each channel runs its own CG recurrence until its
// relative residual |b - A x| / |b| reaches the tolerance (the paper's remark after eq. 2 quotes
// 1e-6 per channel).  Everything runs in float64: the recursive residual of a float32 CG stalls
// near 1e-6 on these systems.
//
// Preconditioner: block Jacobi, the exact inverse of A's 2x2 diagonal blocks
//   D_i = U_i U_i^T + deg_i Id,   deg_i = sum_j w_ij,   det D_i = deg_i (a_i^2 + (1-a_i)^2 + deg_i).
// The paper's remark names a thresholded incomplete Cholesky factor; its triangular solves are
// sequential, while the block diagonal is exact per pixel and parallel.
//
// One iteration is two launches, each followed by a one-workgroup launch that sums the
// per-workgroup partial sums in a fixed order (deterministic) and updates the scalars:
//   spmv:   p = D^-1 r + beta p_old (also at the four neighbours, recomputed from r and p_old),
//           q = A p, partial p.q                               -> alpha = r.z / p.q
//   update: x += alpha p, r -= alpha q, z = D^-1 r, partial r.z and r.r
//                                                              -> beta = r.z_new / r.z, convergence
// (Letting the last workgroup of each launch do that sum instead, behind device-scope fences,
// measured 1.5 - 2x slower per iteration: every workgroup's release fence writes back its
// XCD's L2.)
// The spmv kernel streams: each wave owns a strip of 64 columns (62 stored, lanes 0 and 63 are
// halo) and a band of rows, keeps three rows of p in registers and takes horizontal neighbours
// across lanes with DPP.  Both launches return at once when a device flag says the solve is done,
// so the host can enqueue iterations ahead of the device and poll the flag between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fge_internal.h"

namespace fge {
namespace {

constexpr int kCfThreads = 256;          // 4 waves per workgroup
constexpr int kCfCore = 62;              // stored columns per spmv wave
constexpr int kCfPlainBlocksMax = 1024;  // grid of the pointwise kernels (grid-stride loops)
constexpr int kCfMaxIter = 1000000;

// Scalars of the solve, in the workspace.
struct CfState {
    double bb[3];     // |b_c|^2
    double rz[3];     // r . D^-1 r of the current residual
    double rr[3];     // r . r
    double pq[3];
    double alpha[3];
    double beta[3];
    double tol2[3];   // tol^2 |b_c|^2
    double fin_rr[3]; // |b - A x~|^2 of the stored result x~ (final launch)
    int32_t it[3];    // iterations each channel ran
    int32_t conv[3];  // channel reached its tolerance
    int32_t done;     // every channel converged, or max_iter reached
    int32_t iter;     // iterations run
    int32_t max_iter;
    int32_t breakdown;
};

template <typename T>
__device__ __forceinline__ double ldd(const T *p, size_t i) {
    return static_cast<double>(p[i]);
}

__device__ __forceinline__ double wgt(double a, double b, double omega, double eps) {
    return eps + omega * fabs(a - b);
}

// Lane i receives v from lane i-1 (DPP wave_shr:1) / from lane i+1 (wave_shl:1); lane 0 / 63
// receives 0.  Only used where those lanes are halo.
__device__ __forceinline__ double from_left_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum of v over the workgroup in a fixed order; the result is valid in thread 0.
template <int N>
__device__ void block_sum(double (&v)[N], double *red /* [4][N] in LDS */) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) red[wid * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = ((red[k] + red[N + k]) + red[2 * N + k]) + red[3 * N + k];
}

// Workgroup blockIdx.x's N partial sums into part[blockIdx.x * N ...].
template <int N>
__device__ void block_partial(double (&v)[N], double *part) {
    __shared__ double red[4 * N];
    block_sum<N>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) part[static_cast<size_t>(blockIdx.x) * N + k] = v[k];
}

// In a one-workgroup launch: the totals of nb workgroups' partial sums, valid in thread 0.  Thread
// t sums workgroups t, t + 256, t + 512, ... in that order (four workgroups' loads in flight at a
// time), then the workgroup sums the threads in a fixed tree: the result is deterministic.
template <int N>
__device__ void finish_sum(const double *part, unsigned nb, double (&tot)[N]) {
    __shared__ double red[4 * N];
    double s[N];
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] = 0.0;
    for (unsigned b0 = threadIdx.x; b0 < nb; b0 += 4 * kCfThreads) {
        double v[4][N];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const unsigned b = b0 + t * kCfThreads;
#pragma unroll
            for (int k = 0; k < N; ++k) v[t][k] = b < nb ? part[static_cast<size_t>(b) * N + k] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int k = 0; k < N; ++k) s[k] += v[t][k];
    }
    block_sum<N>(s, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) tot[k] = s[k];
}

// Edge weights of pixel (x, y): left, right, up, down (0 where the neighbour is outside).
struct Edges {
    double a, wl, wr, wu, wd;
};

template <typename T>
__device__ __forceinline__ Edges edges_at(const T *A, int W, int H, int x, int y, double omega,
                                          double eps) {
    // all five loads unconditional (clamped addresses), so they are in flight together
    const size_t i = static_cast<size_t>(y) * W + x;
    const double a = ldd(A, i);
    const double l = ldd(A, x > 0 ? i - 1 : i), r = ldd(A, x < W - 1 ? i + 1 : i);
    const double u = ldd(A, y > 0 ? i - W : i), d = ldd(A, y < H - 1 ? i + W : i);
    Edges e;
    e.a = a;
    e.wl = x > 0 ? wgt(a, l, omega, eps) : 0.0;
    e.wr = x < W - 1 ? wgt(a, r, omega, eps) : 0.0;
    e.wu = y > 0 ? wgt(a, u, omega, eps) : 0.0;
    e.wd = y < H - 1 ? wgt(a, d, omega, eps) : 0.0;
    return e;
}

// z = D^-1 r for the block of a pixel with matte a and degree d.
__device__ __forceinline__ void dinv(double a, double d, double r0, double r1, double *z0,
                                     double *z1) {
    const double u1 = 1.0 - a;
    const double m00 = a * a + d, m01 = a * u1, m11 = u1 * u1 + d;
    const double inv = 1.0 / (d * (a * a + u1 * u1 + d));
    *z0 = (m11 * r0 - m01 * r1) * inv;
    *z1 = (m00 * r1 - m01 * r0) * inv;
}

// Grid of a pointwise launch: its threads walk the image in units of one row segment of
// kCfThreads pixels (so a pixel's row and column cost one division per unit, not per pixel).
unsigned plain_blocks(int W, int H) {
    const long units = static_cast<long>(H) * ((W + kCfThreads - 1) / kCfThreads);
    return static_cast<unsigned>(std::min<long>(units, kCfPlainBlocksMax));
}

// ---- start: x = x0 (zero or the caller's F, B), r = b - A x, z = D^-1 r, p_old = 0 ----------

template <typename T>
__global__ __launch_bounds__(kCfThreads) void cf_init_kernel(const T *__restrict__ I,
                                                             const T *__restrict__ A,
                                                             const T *__restrict__ F0,
                                                             const T *__restrict__ B0, int W,
                                                             int H, double omega, double eps,
                                                             double *__restrict__ x,
                                                             double *__restrict__ r,
                                                             double *__restrict__ p,
                                                             double *part, CfState *st) {
    const size_t n = static_cast<size_t>(W) * H;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // bb, rz, rr per channel
    const int segs = (W + kCfThreads - 1) / kCfThreads, units = H * segs;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int y = u / segs, xx = (u - y * segs) * kCfThreads + static_cast<int>(threadIdx.x);
        if (xx >= W) continue;
        const size_t i = static_cast<size_t>(y) * W + xx;
        const Edges e = edges_at(A, W, H, xx, y, omega, eps);
        const double d = e.wl + e.wr + e.wu + e.wd, u1 = 1.0 - e.a;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double b0 = e.a * ldd(I, c * n + i), b1 = u1 * ldd(I, c * n + i);
            double r0 = b0, r1 = b1, f = 0.0, g = 0.0;
            if (F0) {
                const T *Fc = F0 + c * n, *Bc = B0 + c * n;
                f = ldd(Fc, i);
                g = ldd(Bc, i);
                const double s = e.a * f + u1 * g;
                double af = e.a * s, ag = u1 * s;
                if (xx > 0) { af += e.wl * (f - ldd(Fc, i - 1)); ag += e.wl * (g - ldd(Bc, i - 1)); }
                if (xx < W - 1) { af += e.wr * (f - ldd(Fc, i + 1)); ag += e.wr * (g - ldd(Bc, i + 1)); }
                if (y > 0) { af += e.wu * (f - ldd(Fc, i - W)); ag += e.wu * (g - ldd(Bc, i - W)); }
                if (y < H - 1) { af += e.wd * (f - ldd(Fc, i + W)); ag += e.wd * (g - ldd(Bc, i + W)); }
                r0 -= af;
                r1 -= ag;
            }
            double z0, z1;
            dinv(e.a, d, r0, r1, &z0, &z1);
            x[c * n + i] = f;
            x[(c + 3) * n + i] = g;
            r[c * n + i] = r0;
            r[(c + 3) * n + i] = r1;
            p[c * n + i] = 0.0;
            p[(c + 3) * n + i] = 0.0;
            acc[c] += b0 * b0 + b1 * b1;
            acc[3 + c] += r0 * z0 + r1 * z1;
            acc[6 + c] += r0 * r0 + r1 * r1;
        }
    }
    block_partial<9>(acc, part);
}

__global__ __launch_bounds__(kCfThreads) void cf_init_finish(const double *part, unsigned nb, CfState *st) {
    double tot[9];
    finish_sum<9>(part, nb, tot);
    if (threadIdx.x != 0) return;
    const double tol = st->tol2[0];   // the host stores tol^2 here; scaled per channel now
    int all = 1;
    for (int c = 0; c < 3; ++c) {
        st->bb[c] = tot[c];
        st->rz[c] = tot[3 + c];
        st->rr[c] = tot[6 + c];
        st->tol2[c] = tol * tot[c];
        st->beta[c] = 0.0;
        st->alpha[c] = 0.0;
        st->it[c] = 0;
        st->conv[c] = tot[6 + c] <= st->tol2[c] ? 1 : 0;
        all &= st->conv[c];
    }
    st->iter = 0;
    st->breakdown = 0;
    st->done = all || st->max_iter <= 0;
}

// ---- spmv: p = D^-1 r + beta p_old, q = A p, partial p.q ------------------------------------

// One row of the wave's strip: p at row j of this lane's column, with the weights of its four
// edges and its matte value.
struct CfRow {
    double p[6];
    double a, wl, wr, wu, wd;
};

// The memory reads behind a CfRow: r and the previous direction at (x, j), the matte left and
// right of it.  Issued one row ahead of their use.
struct CfLoad {
    double r[6], o[6];
    double al, ar;
};

template <typename T>
__device__ __forceinline__ void cf_load(const T *__restrict__ A, const double *__restrict__ r,
                                        const double *__restrict__ pold, int W, int H, size_t n,
                                        int x, int j, CfLoad *L) {
    // lanes and rows outside the image read clamped addresses (their p is zeroed in cf_make)
    const int xc = min(max(x, 0), W - 1), jc = min(max(j, 0), H - 1);
    const size_t i = static_cast<size_t>(jc) * W + xc;
    L->al = ldd(A, xc > 0 ? i - 1 : i);
    L->ar = ldd(A, xc < W - 1 ? i + 1 : i);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        L->r[k] = r[k * n + i];
        L->o[k] = pold[k * n + i];
    }
}

// p = D^-1 r + beta p_old at (x, j) from its loads, the matte a there and a_up / a_dn above and
// below (used when has_up / has_dn).  Every lane runs this; outside the image p = 0.
__device__ __forceinline__ void cf_make(const CfLoad &L, int W, int H, int x, int j, double a_up,
                                        double a_dn, bool has_up, bool has_dn, double a,
                                        double omega, double eps, const double (&beta)[3],
                                        CfRow *out) {
    const bool in = x >= 0 && x < W && j >= 0 && j < H;
    out->a = a;
    out->wl = in && x > 0 ? wgt(a, L.al, omega, eps) : 0.0;
    out->wr = in && x < W - 1 ? wgt(a, L.ar, omega, eps) : 0.0;
    out->wu = in && has_up ? wgt(a, a_up, omega, eps) : 0.0;
    out->wd = in && has_dn ? wgt(a, a_dn, omega, eps) : 0.0;
    const double d = out->wl + out->wr + out->wu + out->wd;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double z0 = 0.0, z1 = 0.0;
        if (in) dinv(a, d, L.r[c], L.r[c + 3], &z0, &z1);
        out->p[c] = in ? z0 + beta[c] * L.o[c] : 0.0;
        out->p[c + 3] = in ? z1 + beta[c] * L.o[c + 3] : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kCfThreads) void cf_spmv_kernel(
    const T *__restrict__ A, const double *__restrict__ r, const double *__restrict__ pold,
    double *__restrict__ pnew, double *__restrict__ q, int W, int H, double omega, double eps,
    int rows, int strips_x, int nstrips, int chunk, double *part, CfState *st) {
    if (st->done) return;
    const int lane = threadIdx.x & 63;
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so consecutive
    // logical strips (a band of rows, left to right) are given to the workgroups of one XCD.
    const int lb = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
    const int strip = lb * 4 + (threadIdx.x >> 6);
    double beta[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) beta[c] = st->beta[c];
    double acc[3] = {0.0, 0.0, 0.0};
    if (strip < nstrips) {
        const size_t n = static_cast<size_t>(W) * H;
        const int sx = strip % strips_x, sy = strip / strips_x;
        const int x = sx * kCfCore - 1 + lane;
        const int y0 = sy * rows, y1 = min(H, y0 + rows);
        const bool colv = x >= 0 && x < W;
        const bool core = colv && lane >= 1 && lane <= kCfCore;
        const int xc = min(max(x, 0), W - 1);
        auto acol = [&](int j) {   // matte at (xc, j), j clamped into the image
            return ldd(A, static_cast<size_t>(min(max(j, 0), H - 1)) * W + xc);
        };
        // rows y0-1 (prev) and y0 (cur) first; then each step makes row y+1 from loads issued
        // one step earlier, issues the loads of row y+2, and computes q of row y
        double a_m2 = acol(y0 - 2), a_m1 = acol(y0 - 1), a_0 = acol(y0), a_p1 = acol(y0 + 1);
        CfLoad L0, L1;
        cf_load(A, r, pold, W, H, n, x, y0 - 1, &L0);
        cf_load(A, r, pold, W, H, n, x, y0, &L1);
        CfRow prev, cur, next;
        cf_make(L0, W, H, x, y0 - 1, a_m2, a_0, y0 - 1 > 0, y0 < H, a_m1, omega, eps, beta, &prev);
        cf_make(L1, W, H, x, y0, a_m1, a_p1, y0 > 0, y0 + 1 < H, a_0, omega, eps, beta, &cur);
        cf_load(A, r, pold, W, H, n, x, y0 + 1, &L0);   // row y0 + 1
        double a_j = a_p1, a_n = acol(y0 + 2);           // matte of rows y+1, y+2
        for (int y = y0; y < y1; ++y) {
            CfLoad Ln;
            cf_load(A, r, pold, W, H, n, x, y + 2, &Ln);
            const double a_nn = acol(y + 3);
            cf_make(L0, W, H, x, y + 1, cur.a, a_n, true, y + 2 < H, a_j, omega, eps, beta, &next);
            L0 = Ln;
            a_j = a_n;
            a_n = a_nn;
            const double u1 = 1.0 - cur.a;
            double qv[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double f = cur.p[c], g = cur.p[c + 3];
                const double fl = from_left_d(f), fr = from_right_d(f);
                const double gl = from_left_d(g), gr = from_right_d(g);
                const double s = cur.a * f + u1 * g;
                qv[c] = cur.a * s + cur.wl * (f - fl) + cur.wr * (f - fr) + cur.wu * (f - prev.p[c]) +
                        cur.wd * (f - next.p[c]);
                qv[c + 3] = u1 * s + cur.wl * (g - gl) + cur.wr * (g - gr) +
                            cur.wu * (g - prev.p[c + 3]) + cur.wd * (g - next.p[c + 3]);
            }
            if (core) {
                const size_t i = static_cast<size_t>(y) * W + x;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pnew[c * n + i] = cur.p[c];
                    pnew[(c + 3) * n + i] = cur.p[c + 3];
                    q[c * n + i] = qv[c];
                    q[(c + 3) * n + i] = qv[c + 3];
                    acc[c] += cur.p[c] * qv[c] + cur.p[c + 3] * qv[c + 3];
                }
            }
            prev = cur;
            cur = next;
        }
    }
    block_partial<3>(acc, part);
}

__global__ __launch_bounds__(kCfThreads) void cf_spmv_finish(const double *part, unsigned nb, CfState *st) {
    if (st->done) return;
    double tot[3];
    finish_sum<3>(part, nb, tot);
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 3; ++c) {
        st->pq[c] = tot[c];
        if (st->conv[c]) {
            st->alpha[c] = 0.0;
        } else if (!(tot[c] > 0.0)) {   // A is not positive definite on this direction
            st->alpha[c] = 0.0;
            st->conv[c] = 1;
            st->breakdown = 1;
        } else {
            st->alpha[c] = st->rz[c] / tot[c];
        }
    }
}

// ---- update: x += alpha p, r -= alpha q, z = D^-1 r, partial r.z and r.r --------------------

template <typename T>
__global__ __launch_bounds__(kCfThreads) void cf_update_kernel(
    const T *__restrict__ A, double *__restrict__ x, const double *__restrict__ p,
    double *__restrict__ r, const double *__restrict__ q, int W, int H, double omega, double eps,
    double *part, CfState *st) {
    if (st->done) return;
    const size_t n = static_cast<size_t>(W) * H;
    double al[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) al[c] = st->alpha[c];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int segs = (W + kCfThreads - 1) / kCfThreads, units = H * segs;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int y = u / segs, xx = (u - y * segs) * kCfThreads + static_cast<int>(threadIdx.x);
        if (xx >= W) continue;
        const size_t i = static_cast<size_t>(y) * W + xx;
        const Edges e = edges_at(A, W, H, xx, y, omega, eps);
        const double d = e.wl + e.wr + e.wu + e.wd;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i0 = c * n + i, i1 = (c + 3) * n + i;
            x[i0] += al[c] * p[i0];
            x[i1] += al[c] * p[i1];
            const double r0 = r[i0] - al[c] * q[i0], r1 = r[i1] - al[c] * q[i1];
            r[i0] = r0;
            r[i1] = r1;
            double z0, z1;
            dinv(e.a, d, r0, r1, &z0, &z1);
            acc[c] += r0 * z0 + r1 * z1;
            acc[3 + c] += r0 * r0 + r1 * r1;
        }
    }
    block_partial<6>(acc, part);
}

__global__ __launch_bounds__(kCfThreads) void cf_update_finish(const double *part, unsigned nb, CfState *st) {
    if (st->done) return;
    double tot[6];
    finish_sum<6>(part, nb, tot);
    if (threadIdx.x != 0) return;
    int all = 1;
    for (int c = 0; c < 3; ++c) {
        if (!st->conv[c]) {
            st->it[c] += 1;
            st->beta[c] = tot[c] / st->rz[c];
            st->rz[c] = tot[c];
            st->rr[c] = tot[3 + c];
            if (tot[3 + c] <= st->tol2[c]) st->conv[c] = 1;
        }
        if (st->conv[c]) st->beta[c] = 0.0;
        all &= st->conv[c];
    }
    st->iter += 1;
    st->done = all || st->iter >= st->max_iter;
}

// ---- result: F, B = x rounded to the storage type; |b - A x~|^2 of that rounded result -------

template <typename T>
__global__ __launch_bounds__(kCfThreads) void cf_final_kernel(const T *__restrict__ I,
                                                              const T *__restrict__ A,
                                                              const double *__restrict__ x,
                                                              T *__restrict__ F, T *__restrict__ B,
                                                              int W, int H, double omega,
                                                              double eps, double *part,
                                                              CfState *st) {
    const size_t n = static_cast<size_t>(W) * H;
    auto rd = [&](size_t k) { return static_cast<double>(static_cast<T>(x[k])); };
    double acc[3] = {0, 0, 0};
    const int segs = (W + kCfThreads - 1) / kCfThreads, units = H * segs;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int y = u / segs, xx = (u - y * segs) * kCfThreads + static_cast<int>(threadIdx.x);
        if (xx >= W) continue;
        const size_t i = static_cast<size_t>(y) * W + xx;
        const Edges e = edges_at(A, W, H, xx, y, omega, eps);
        const double u1 = 1.0 - e.a;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i0 = c * n + i, i1 = (c + 3) * n + i;
            const double f = rd(i0), g = rd(i1);
            const double s = e.a * f + u1 * g;
            double af = e.a * s, ag = u1 * s;
            if (xx > 0) { af += e.wl * (f - rd(i0 - 1)); ag += e.wl * (g - rd(i1 - 1)); }
            if (xx < W - 1) { af += e.wr * (f - rd(i0 + 1)); ag += e.wr * (g - rd(i1 + 1)); }
            if (y > 0) { af += e.wu * (f - rd(i0 - W)); ag += e.wu * (g - rd(i1 - W)); }
            if (y < H - 1) { af += e.wd * (f - rd(i0 + W)); ag += e.wd * (g - rd(i1 + W)); }
            const double v = ldd(I, i0);
            const double r0 = e.a * v - af, r1 = u1 * v - ag;
            acc[c] += r0 * r0 + r1 * r1;
            F[c * n + i] = static_cast<T>(x[i0]);
            B[c * n + i] = static_cast<T>(x[i1]);
        }
    }
    block_partial<3>(acc, part);
}

__global__ __launch_bounds__(kCfThreads) void cf_final_finish(const double *part, unsigned nb, CfState *st) {
    double tot[3];
    finish_sum<3>(part, nb, tot);
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 3; ++c) st->fin_rr[c] = tot[c];
}

// ---- host side -------------------------------------------------------------------------------

struct CfLayout {
    size_t state, part, vec[5], total;   // vec: x, r, p0, p1, q (6 planes of doubles each)
};

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

int spmv_rows(int W, int H) {
    // Rows per wave strip.  Measured at 1024 x 768 (float32 storage, microseconds per iteration
    // of both launches): 4 rows 77.7, 8 rows 72.9, 16 rows 71.3, 32 rows 78.1.
    (void)W;
    return std::min(H, 16);
}

int spmv_blocks(int W, int H, int *rows, int *strips_x, int *nstrips, int *chunk) {
    *rows = spmv_rows(W, H);
    *strips_x = (W + kCfCore - 1) / kCfCore;
    *nstrips = *strips_x * ((H + *rows - 1) / *rows);
    const int groups = (*nstrips + 3) / 4;
    *chunk = (groups + 7) / 8;
    return 8 * *chunk;
}

CfLayout cf_layout(int W, int H) {
    CfLayout L;
    const size_t n = static_cast<size_t>(W) * H;
    int rows, sx, ns, ch;
    const size_t blocks = std::max<size_t>(spmv_blocks(W, H, &rows, &sx, &ns, &ch), kCfPlainBlocksMax);
    L.state = 0;
    L.part = align256(sizeof(CfState));
    size_t off = align256(L.part + blocks * 9 * sizeof(double));
    for (int k = 0; k < 5; ++k) {
        L.vec[k] = off;
        off = align256(off + 6 * n * sizeof(double));
    }
    L.total = off;
    return L;
}

template <typename T>
fge_status cf_run(const void *I, const void *A, int W, int H, const fge_cf_params &p, void *F,
                  void *B, char *ws, hipStream_t s, fge_cf_info *info) {
    const CfLayout L = cf_layout(W, H);
    const size_t n = static_cast<size_t>(W) * H;
    CfState *st = reinterpret_cast<CfState *>(ws + L.state);
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *x = reinterpret_cast<double *>(ws + L.vec[0]);
    double *r = reinterpret_cast<double *>(ws + L.vec[1]);
    double *pb[2] = {reinterpret_cast<double *>(ws + L.vec[2]),
                     reinterpret_cast<double *>(ws + L.vec[3])};
    double *q = reinterpret_cast<double *>(ws + L.vec[4]);
    const T *It = static_cast<const T *>(I), *At = static_cast<const T *>(A);
    const int max_iter = p.max_iter > 0 ? p.max_iter : 20000;

    // Scalars: counters zero, tol^2 in tol2[0] (the start kernel scales it by |b_c|^2).
    CfState init{};
    init.tol2[0] = p.tol * p.tol;
    init.max_iter = max_iter;
    int32_t *host = nullptr;   // pinned: two polling slots (done, iter) and the final state
    if (hipHostMalloc(reinterpret_cast<void **>(&host), 4 * sizeof(int32_t) + sizeof(CfState),
                      hipHostMallocDefault) != hipSuccess)
        return FGE_ENOMEM;
    hipEvent_t ev[2] = {nullptr, nullptr}, tev[2] = {nullptr, nullptr};
    fge_status ret = FGE_OK;
    auto fail = [&](fge_status e) { ret = e; };
    CfState *hst = reinterpret_cast<CfState *>(host + 4);
    *hst = init;
    if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&tev[0]) != hipSuccess || hipEventCreate(&tev[1]) != hipSuccess) {
        fail(FGE_EHIP);
    }
    const unsigned pb_blocks = plain_blocks(W, H);
    int rows, strips_x, nstrips, chunk;
    const unsigned sp_blocks = static_cast<unsigned>(spmv_blocks(W, H, &rows, &strips_x, &nstrips, &chunk));
    const double om = p.omega, ep = p.eps;
    const T *F0 = p.warm_start ? static_cast<const T *>(F) : nullptr;
    const T *B0 = p.warm_start ? static_cast<const T *>(B) : nullptr;
    int enq = 0;
    if (ret == FGE_OK) {
        if (hipMemcpyAsync(st, hst, sizeof(CfState), hipMemcpyHostToDevice, s) != hipSuccess) fail(FGE_EHIP);
    }
    if (ret == FGE_OK && hipEventRecord(tev[0], s) != hipSuccess) fail(FGE_EHIP);
    if (ret == FGE_OK) {
        cf_init_kernel<T><<<pb_blocks, kCfThreads, 0, s>>>(It, At, F0, B0, W, H, om, ep, x, r, pb[0],
                                                           part, st);
        cf_init_finish<<<1, kCfThreads, 0, s>>>(part, pb_blocks, st);
        if (hipGetLastError() != hipSuccess) fail(FGE_EHIP);
    }
    // Iterations in chunks of growing length; after each chunk the (done, iter) words are copied
    // to a pinned slot behind an event.  The host waits for the previous chunk's event only, so
    // the device always has the next chunk queued; launches after the flag is set return at once.
    int slot = 0, prev = -1, len = 4;
    while (ret == FGE_OK && enq < max_iter) {
        const int k = std::min(len, max_iter - enq);
        for (int t = 0; t < k && ret == FGE_OK; ++t, ++enq) {
            double *po = pb[enq & 1], *pn = pb[(enq + 1) & 1];
            cf_spmv_kernel<T><<<sp_blocks, kCfThreads, 0, s>>>(At, r, po, pn, q, W, H, om, ep, rows,
                                                               strips_x, nstrips, chunk, part, st);
            cf_spmv_finish<<<1, kCfThreads, 0, s>>>(part, sp_blocks, st);
            cf_update_kernel<T><<<pb_blocks, kCfThreads, 0, s>>>(At, x, pn, r, q, W, H, om, ep, part,
                                                                 st);
            cf_update_finish<<<1, kCfThreads, 0, s>>>(part, pb_blocks, st);
            if (hipGetLastError() != hipSuccess) fail(FGE_EHIP);
        }
        if (ret != FGE_OK) break;
        if (hipMemcpyAsync(host + 2 * slot, &st->done, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipEventRecord(ev[slot], s) != hipSuccess) {
            fail(FGE_EHIP);
            break;
        }
        if (prev >= 0) {
            if (hipEventSynchronize(ev[prev]) != hipSuccess) {
                fail(FGE_EHIP);
                break;
            }
            if (host[2 * prev]) break;
        }
        prev = slot;
        slot ^= 1;
        len = std::min(len * 2, 64);
    }
    if (ret == FGE_OK) {
        cf_final_kernel<T><<<pb_blocks, kCfThreads, 0, s>>>(It, At, x, static_cast<T *>(F),
                                                            static_cast<T *>(B), W, H, om, ep, part,
                                                            st);
        cf_final_finish<<<1, kCfThreads, 0, s>>>(part, pb_blocks, st);
        if (hipGetLastError() != hipSuccess || hipEventRecord(tev[1], s) != hipSuccess ||
            hipMemcpyAsync(hst, st, sizeof(CfState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            fail(FGE_EHIP);
    }
    float dev_ms = 0.0f;
    if (ret == FGE_OK && hipEventElapsedTime(&dev_ms, tev[0], tev[1]) != hipSuccess) fail(FGE_EHIP);
    if (ret == FGE_OK && info) {
        int itmax = 0;
        info->converged = hst->conv[0] && hst->conv[1] && hst->conv[2] && !hst->breakdown;
        for (int c = 0; c < 3; ++c) {
            info->channel_iterations[c] = hst->it[c];
            itmax = std::max(itmax, static_cast<int>(hst->it[c]));
            const double bb = hst->bb[c];
            info->rel_residual[c] = bb > 0.0 ? std::sqrt(hst->fin_rr[c] / bb) : 0.0;
            info->recursive_rel_residual[c] = bb > 0.0 ? std::sqrt(hst->rr[c] / bb) : 0.0;
        }
        info->iterations = itmax;
        info->breakdown = hst->breakdown;
        info->device_ms = dev_ms;
    }
    if (ret != FGE_OK) (void)hipStreamSynchronize(s);   // no queued copy may still target `host`
    for (hipEvent_t e : {ev[0], ev[1], tev[0], tev[1]})
        if (e) (void)hipEventDestroy(e);
    (void)hipHostFree(host);
    return ret;
}

}  // namespace
}  // namespace fge

extern "C" {

void fge_cf_default_params(fge_cf_params *p) {
    if (!p) return;
    *p = fge_cf_params{};
    p->size = sizeof(fge_cf_params);
    p->omega = 1.0;
    p->eps = 5e-3;
    p->tol = 1e-6;
    p->max_iter = 20000;
    p->storage = FGE_F32;
    p->warm_start = 0;
}

size_t fge_cf_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1 || H > fge::kMaxSide || W > fge::kMaxSide) return 0;
    return fge::cf_layout(W, H).total;
}

fge_status fge_closed_form(const void *I, const void *alpha, int32_t H, int32_t W,
                           const fge_cf_params *p, void *F, void *B, void *workspace,
                           size_t workspace_bytes, void *stream, fge_cf_info *info) {
    fge_cf_params def;
    if (!p) {
        fge_cf_default_params(&def);
        p = &def;
    }
    if (p->size != sizeof(fge_cf_params)) return FGE_EINVAL;
    if (H < 1 || W < 1 || H > fge::kMaxSide || W > fge::kMaxSide) return FGE_EINVAL;
    if (static_cast<long long>(H) * W < 2) return FGE_EINVAL;
    if (!(p->eps > 0.0) || !(p->omega >= 0.0) || !std::isfinite(p->eps) || !std::isfinite(p->omega))
        return FGE_EINVAL;
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return FGE_EINVAL;
    if (p->max_iter < 0 || p->max_iter > fge::kCfMaxIter) return FGE_EINVAL;
    if (p->storage != FGE_F32 && p->storage != FGE_F16 && p->storage != FGE_F64) return FGE_EINVAL;
    if (!I || !alpha || !F || !B) return FGE_EINVAL;
    const int elem = p->storage == FGE_F16 ? 2 : (p->storage == FGE_F64 ? 8 : 4);
    if (fge::outputs_alias(I, alpha, F, B, W, H, elem, workspace, workspace_bytes)) return FGE_EINVAL;
    const size_t need = fge::cf_layout(W, H).total;
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return FGE_EWORKSPACE;
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->storage == FGE_F16)
        return fge::cf_run<_Float16>(I, alpha, W, H, *p, F, B, ws, s, info);
    if (p->storage == FGE_F64)
        return fge::cf_run<double>(I, alpha, W, H, *p, F, B, ws, s, info);
    return fge::cf_run<float>(I, alpha, W, H, *p, F, B, ws, s, info);
}

}  // extern "C"
