// Reporting and layout kernels (C ABI in include/fge.h): the energy of a result and its
// compositing residual, reduced on the device, and conversions between interleaved 8-bit or
// float images and the planar storage the estimator works on.
//
// Energy (the quadratic whose per-pixel stationarity conditions are the 2x2 systems of eq. 9):
//   E = sum_i sum_c (a_i F_i^c + (1 - a_i) B_i^c - I_i^c)^2
//     + sum over undirected in-bounds 4-neighbour edges {i, j}, each once, of
//       (eps_r + omega |a_i - a_j|) sum_c [(F_i^c - F_j^c)^2 + (B_i^c - B_j^c)^2].
// Every pixel adds its data term and the edges to its right and lower neighbours.  Terms are
// formed and summed in float64: per thread, per block (fixed tree order in LDS), then over the
// blocks' partial sums by one workgroup in a fixed order, so the result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fge_internal.h"

namespace fge {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocksMax = 2048;

template <typename T>
__device__ __forceinline__ double ld(const T *p, size_t i) {
    return static_cast<double>(static_cast<float>(p[i]));
}

// Partial sums of one block: [0] data term, [1] smoothness term, [2] sum of |residual| over
// fractional pixels (0 < a < 1), [3] number of fractional pixels, [4] max |residual| there.
// The energy is that of a w x h level.  I and alpha are W x H and F and B are fw x fh; both are
// read through the nearest map onto the level (source index (x W / w, y H / h), likewise with fw,
// fh; the identity when the sizes agree), so the state of the previous level can be evaluated as
// it stands after the resize.  Threads walk the level in row segments of kRedThreads pixels (one
// division per segment).  A non-null `stop` that holds a non-zero value turns the launch into a
// no-op.
template <typename T, typename TF>
__global__ __launch_bounds__(kRedThreads) void energy_partial_kernel(
    const T *I, const T *A, int W, int H, const TF *F, const TF *B, int fw, int fh, int w, int h,
    float omega, float eps, const int *stop, double *part) {
    if (stop && *stop) return;
    const size_t nf = static_cast<size_t>(fw) * fh, nI = static_cast<size_t>(W) * H;
    const bool same = W == w && H == h, fsame = fw == w && fh == h;
    auto src = [&](int xx, int yy) {
        return same ? static_cast<size_t>(yy) * w + xx
                    : static_cast<size_t>(yy * H / h) * W + xx * W / w;
    };
    auto fsrc = [&](int xx, int yy) {
        return fsame ? static_cast<size_t>(yy) * w + xx
                     : static_cast<size_t>(yy * fh / h) * fw + xx * fw / w;
    };
    double data = 0.0, smooth = 0.0, rsum = 0.0, rcnt = 0.0, rmax = 0.0;
    const int segs = (w + kRedThreads - 1) / kRedThreads, units = h * segs;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int y = u / segs, x = (u - y * segs) * kRedThreads + static_cast<int>(threadIdx.x);
        if (x >= w) continue;
        const size_t ps = src(x, y), pf = fsrc(x, y);
        const double a = ld(A, ps);
        const bool frac = a > 0.0 && a < 1.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t q = c * nf + pf;
            const double r = a * ld(F, q) + (1.0 - a) * ld(B, q) - ld(I, c * nI + ps);
            data += r * r;
            if (frac) {
                rsum += fabs(r);
                rmax = fmax(rmax, fabs(r));
            }
        }
        if (frac) rcnt += 1.0;
        if (x + 1 < w) {
            const double s = static_cast<double>(eps) + static_cast<double>(omega) * fabs(a - ld(A, src(x + 1, y)));
            const size_t pr = fsrc(x + 1, y);
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double df = ld(F, c * nf + pf) - ld(F, c * nf + pr);
                const double db = ld(B, c * nf + pf) - ld(B, c * nf + pr);
                d += df * df + db * db;
            }
            smooth += s * d;
        }
        if (y + 1 < h) {
            const double s = static_cast<double>(eps) + static_cast<double>(omega) * fabs(a - ld(A, src(x, y + 1)));
            const size_t pd = fsrc(x, y + 1);
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double df = ld(F, c * nf + pf) - ld(F, c * nf + pd);
                const double db = ld(B, c * nf + pf) - ld(B, c * nf + pd);
                d += df * df + db * db;
            }
            smooth += s * d;
        }
    }
    __shared__ double red[5][kRedThreads];
    red[0][threadIdx.x] = data;
    red[1][threadIdx.x] = smooth;
    red[2][threadIdx.x] = rsum;
    red[3][threadIdx.x] = rcnt;
    red[4][threadIdx.x] = rmax;
    __syncthreads();
    for (int half = kRedThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + half]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) part[static_cast<size_t>(blockIdx.x) * 5 + threadIdx.x] = red[threadIdx.x][0];
}

// out[0] = E, [1] data term, [2] smoothness term, [3] mean |residual| over fractional pixels,
// [4] max |residual| there, [5] number of fractional pixels.
__device__ __forceinline__ void energy_total(const double *part, int nb, double *out) {
    __shared__ double red[5][kRedThreads];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += part[static_cast<size_t>(b) * 5 + k];
        acc[4] = fmax(acc[4], part[static_cast<size_t>(b) * 5 + 4]);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int half = kRedThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + half]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0] + red[1][0];
        out[1] = red[0][0];
        out[2] = red[1][0];
        out[3] = red[3][0] > 0.0 ? red[2][0] / red[3][0] : 0.0;
        out[4] = red[4][0];
        out[5] = red[3][0];
    }
}

__global__ __launch_bounds__(kRedThreads) void energy_final_kernel(const double *part, int nb,
                                                                   const int *stop, double *out) {
    if (stop && *stop) return;
    energy_total(part, nb, out);
}

// energy_final_kernel's total, then the stop rule of the level loop tested after every sweep:
// after sweep k of a level (k = 0: the resized start) record the count and stop when the energy
// changed by at most tol times its value before the sweep, or k reached kmax.  One launch instead
// of a total and a one-thread check.
__global__ __launch_bounds__(kRedThreads) void energy_check_kernel(const double *part, int nb,
                                                                   double *out, double *eprev,
                                                                   int *stop, int *count,
                                                                   double tol, int k, int kmax) {
    if (*stop) return;
    energy_total(part, nb, out);
    if (threadIdx.x == 0) {
        const double e = out[0];
        if (k > 0) {
            count[0] = k;
            if (fabs(eprev[0] - e) <= tol * eprev[0] || k >= kmax) stop[0] = 1;
        }
        eprev[0] = e;
    }
}

// energy_final_kernel's total plus the convergence form's stop rule (PassCtl).  out is host
// memory: out[6] = seq is written after the six values, behind a system-scope fence, so the host
// can poll it.
__global__ __launch_bounds__(kRedThreads) void pass_final_kernel(const double *part, int nb,
                                                                 double *out, PassCtl *ctl, int m,
                                                                 double tol, double seq) {
    if (m > 1 && ctl->stop) return;
    __shared__ double red[2][kRedThreads];
    double acc[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
        acc[0] += part[static_cast<size_t>(b) * 5];
        acc[1] += part[static_cast<size_t>(b) * 5 + 1];
    }
    red[0][threadIdx.x] = acc[0];
    red[1][threadIdx.x] = acc[1];
    __syncthreads();
    for (int half = kRedThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
            red[0][threadIdx.x] += red[0][threadIdx.x + half];
            red[1][threadIdx.x] += red[1][threadIdx.x + half];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = red[0][0] + red[1][0];
        out[0] = e;
        out[1] = red[0][0];
        out[2] = red[1][0];
        out[3] = out[4] = out[5] = 0.0;
        if (m == 1) {
            ctl->e_prev = e;
            ctl->stop = 0;
        } else if (fabs(ctl->e_prev - e) <= tol * ctl->e_prev) {
            ctl->stop = 1;
        } else {
            ctl->e_prev = e;
        }
        __threadfence_system();
        reinterpret_cast<volatile double *>(out)[6] = seq;
    }
}

// ---- quality measures and compositing -------------------------------------------------------
//
// The paper's error measures of a foreground estimate F against a reference G (Section IV,
// "Error Measures"): over the translucent pixels 0 < a_i < 1 of the reference matte, weighted by
// a_i, SAD = sum a_i |F_i - G_i|_1, MSE = sum a_i |F_i - G_i|_2^2 and
// GRAD = sum a_i |grad F_i - grad G_i|_2^2, the gradients from first-order Gaussian derivative
// filters.  The filter is the sampled Gaussian of
// radius int(4 sigma + 0.5) normalised to sum 1; the x derivative at pixel (x, y) is
// sum_a phi(a) sum_b (b / sigma^2) phi(b) D(x + b, y + a), the y derivative likewise with the
// roles swapped, D = F - G (the filters are linear), with mirrored borders (d c b a | a b c d).
// Everything in float64.

constexpr int kGradMaxR = 16;

struct GradFilter {
    int r;
    double phi[2 * kGradMaxR + 1];   // phi[r + j]: normalised Gaussian at offset j
    double der[2 * kGradMaxR + 1];   // der[r + j] = (j / sigma^2) phi[r + j]
};

__device__ __forceinline__ int mirror(int i, int n) {
    const int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void quality_partial_kernel(const T *F, const T *G,
                                                                      const T *A, int w, int h,
                                                                      GradFilter K, double *part) {
    const size_t n = static_cast<size_t>(w) * h;
    double sad = 0.0, mse = 0.0, grad = 0.0, cnt = 0.0;
    const int r = K.r;
    for (size_t p = static_cast<size_t>(blockIdx.x) * kRedThreads + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kRedThreads) {
        const double a = ld(A, p);
        if (!(a > 0.0 && a < 1.0)) continue;
        const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<size_t>(y) * w);
        double s1 = 0.0, s2 = 0.0, g2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const T *Fc = F + c * n, *Gc = G + c * n;
            const double d = ld(Fc, p) - ld(Gc, p);
            s1 += fabs(d);
            s2 += d * d;
            double gx = 0.0, gy = 0.0;
            for (int dy = -r; dy <= r; ++dy) {
                const size_t row = static_cast<size_t>(mirror(y + dy, h)) * w;
                double sx = 0.0, ss = 0.0;
                for (int dx = -r; dx <= r; ++dx) {
                    const size_t q = row + mirror(x + dx, w);
                    const double v = ld(Fc, q) - ld(Gc, q);
                    sx += K.der[r + dx] * v;
                    ss += K.phi[r + dx] * v;
                }
                gx += K.phi[r + dy] * sx;
                gy += K.der[r + dy] * ss;
            }
            g2 += gx * gx + gy * gy;
        }
        sad += a * s1;
        mse += a * s2;
        grad += a * g2;
        cnt += 1.0;
    }
    __shared__ double red[4][kRedThreads];
    red[0][threadIdx.x] = sad;
    red[1][threadIdx.x] = mse;
    red[2][threadIdx.x] = grad;
    red[3][threadIdx.x] = cnt;
    __syncthreads();
    for (int half = kRedThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[static_cast<size_t>(blockIdx.x) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// The same measures, tiled (radius up to kQMaxR): a workgroup takes a kQTx x kQTy tile, loads
// D = F - G of the tile plus an r-pixel mirrored ring into LDS one channel at a time, filters the
// rows (derivative and smoothing filter in x), then the columns (smoothing and derivative in y),
// so a pixel costs 4 (2r + 1) multiply-adds per channel instead of 2 (2r + 1)^2 loads and
// multiply-adds.  Same taps, same float64, another summation order.  One partial (4 sums) per
// tile, reduced in a fixed order.
constexpr int kQTx = 64, kQTy = 16, kQThreads = 256, kQMaxR = 8;
constexpr int kQRw = kQTx + 2 * kQMaxR, kQRh = kQTy + 2 * kQMaxR;
constexpr int kQPx = kQTx * kQTy / kQThreads;   // output pixels per thread

template <typename T>
__global__ __launch_bounds__(kQThreads) void quality_tile_kernel(const T *F, const T *G, const T *A,
                                                                 int w, int h, GradFilter K,
                                                                 double *part) {
    __shared__ double sd[kQRh * kQRw];    // D over the region (row stride RW)
    __shared__ double sx[kQRh * kQTx];    // rows filtered with the derivative
    __shared__ double ss[kQRh * kQTx];    // rows filtered with the smoothing filter
    __shared__ double red[4][kQThreads];
    const int r = K.r, RW = kQTx + 2 * r, RH = kQTy + 2 * r;
    const int tx0 = blockIdx.x * kQTx, ty0 = blockIdx.y * kQTy;
    const int tid = threadIdx.x;
    const size_t n = static_cast<size_t>(w) * h;
    double s1[kQPx] = {}, s2[kQPx] = {}, g2[kQPx] = {};
    for (int c = 0; c < 3; ++c) {
        const T *Fc = F + c * n, *Gc = G + c * n;
        __syncthreads();   // the previous channel's reads of sd, sx, ss are done
        for (int i = tid; i < RW * RH; i += kQThreads) {
            const int ry = i / RW, rx = i - ry * RW;
            const size_t q = static_cast<size_t>(mirror(ty0 - r + ry, h)) * w + mirror(tx0 - r + rx, w);
            sd[i] = ld(Fc, q) - ld(Gc, q);
        }
        __syncthreads();
        for (int i = tid; i < kQTx * RH; i += kQThreads) {
            const int ry = i / kQTx, ox = i - ry * kQTx;
            const double *row = sd + ry * RW + ox;
            double d = 0.0, p = 0.0;
            for (int j = 0; j <= 2 * r; ++j) {
                d += K.der[j] * row[j];
                p += K.phi[j] * row[j];
            }
            sx[i] = d;
            ss[i] = p;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kQPx; ++k) {
            const int q = tid + k * kQThreads, oy = q / kQTx, ox = q - oy * kQTx;
            double gx = 0.0, gy = 0.0;
            for (int j = 0; j <= 2 * r; ++j) {
                gx += K.phi[j] * sx[(oy + j) * kQTx + ox];
                gy += K.der[j] * ss[(oy + j) * kQTx + ox];
            }
            g2[k] += gx * gx + gy * gy;
            const double d = sd[(oy + r) * RW + ox + r];
            s1[k] += fabs(d);
            s2[k] += d * d;
        }
    }
    double sad = 0.0, mse = 0.0, grad = 0.0, cnt = 0.0;
#pragma unroll
    for (int k = 0; k < kQPx; ++k) {
        const int q = tid + k * kQThreads, x = tx0 + q % kQTx, y = ty0 + q / kQTx;
        if (x >= w || y >= h) continue;
        const double a = ld(A, static_cast<size_t>(y) * w + x);
        if (!(a > 0.0 && a < 1.0)) continue;
        sad += a * s1[k];
        mse += a * s2[k];
        grad += a * g2[k];
        cnt += 1.0;
    }
    red[0][tid] = sad;
    red[1][tid] = mse;
    red[2][tid] = grad;
    red[3][tid] = cnt;
    __syncthreads();
    for (int half = kQThreads / 2; half > 0; half >>= 1) {
        if (tid < half)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + half];
        __syncthreads();
    }
    if (tid < 4) part[(static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * 4 + tid] = red[tid][0];
}

__global__ __launch_bounds__(kRedThreads) void quality_final_kernel(const double *part, int nb,
                                                                    double *out) {
    __shared__ double red[4][kRedThreads];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += part[static_cast<size_t>(b) * 4 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int half = kRedThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

// C = a F + (1 - a) B in float64, each product and the sum rounded once (no contraction), then
// converted to T.
template <typename T>
__global__ __launch_bounds__(256) void composite_kernel(const T *F, const T *A, const T *B, T *C,
                                                        size_t n) {
    const size_t p = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= n) return;
    const double a = ld(A, p);
    const double b = __dadd_rn(1.0, -a);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = __dadd_rn(__dmul_rn(a, ld(F, c * n + p)), __dmul_rn(b, ld(B, c * n + p)));
        C[c * n + p] = static_cast<T>(v);
    }
}

// ---- layout --------------------------------------------------------------------------------

template <typename S>
__device__ __forceinline__ float to_unit(S v) {
    if constexpr (sizeof(S) == 1) return static_cast<float>(v) / 255.0f;
    else return static_cast<float>(v);
}

template <typename D>
__device__ __forceinline__ D from_unit(float v) {
    if constexpr (sizeof(D) == 1) {
        const float c = fminf(fmaxf(v, 0.0f), 1.0f) * 255.0f;
        return static_cast<D>(__float2int_rn(c));
    } else {
        return static_cast<D>(v);
    }
}

// Interleaved H x W x C (C = 3 or 4) -> planes: 3 colour planes, and the 4th channel as alpha.
template <typename S, typename D>
__global__ __launch_bounds__(256) void hwc_to_planar_kernel(const S *src, int C, size_t n,
                                                            D *planes, D *alpha) {
    const size_t p = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= n) return;
    const S *px = src + p * C;
#pragma unroll
    for (int c = 0; c < 3; ++c) planes[c * n + p] = from_unit<D>(to_unit(px[c]));
    if (C == 4 && alpha) alpha[p] = from_unit<D>(to_unit(px[3]));
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void planar_to_hwc_kernel(const S *planes, size_t n, D *dst) {
    const size_t p = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[p * 3 + c] = from_unit<D>(to_unit(planes[c * n + p]));
}

template <typename S>
int launch_h2p_src(const void *src, int C, size_t n, int dst_dtype, void *planes, void *alpha,
                   hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    const S *sp = static_cast<const S *>(src);
    switch (dst_dtype) {
        case FGE_F32:
            hipLaunchKernelGGL((hwc_to_planar_kernel<S, float>), grid, dim3(256), 0, s, sp, C, n,
                               static_cast<float *>(planes), static_cast<float *>(alpha));
            break;
        case FGE_F16:
            hipLaunchKernelGGL((hwc_to_planar_kernel<S, _Float16>), grid, dim3(256), 0, s, sp, C, n,
                               static_cast<_Float16 *>(planes), static_cast<_Float16 *>(alpha));
            break;
        default:
            hipLaunchKernelGGL((hwc_to_planar_kernel<S, uint8_t>), grid, dim3(256), 0, s, sp, C, n,
                               static_cast<uint8_t *>(planes), static_cast<uint8_t *>(alpha));
            break;
    }
    return static_cast<int>(hipGetLastError());
}

template <typename S>
int launch_p2h_src(const void *src, size_t n, int dst_dtype, void *dst, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    const S *sp = static_cast<const S *>(src);
    switch (dst_dtype) {
        case FGE_F32:
            hipLaunchKernelGGL((planar_to_hwc_kernel<S, float>), grid, dim3(256), 0, s, sp, n,
                               static_cast<float *>(dst));
            break;
        case FGE_F16:
            hipLaunchKernelGGL((planar_to_hwc_kernel<S, _Float16>), grid, dim3(256), 0, s, sp, n,
                               static_cast<_Float16 *>(dst));
            break;
        default:
            hipLaunchKernelGGL((planar_to_hwc_kernel<S, uint8_t>), grid, dim3(256), 0, s, sp, n,
                               static_cast<uint8_t *>(dst));
            break;
    }
    return static_cast<int>(hipGetLastError());
}

bool dtype_ok(int d) { return d == FGE_F32 || d == FGE_F16 || d == FGE_U8; }

}  // namespace

int energy_blocks(int w, int h) {
    const size_t n = static_cast<size_t>(w) * h;
    const size_t b = (n + kRedThreads - 1) / kRedThreads;
    return static_cast<int>(b < static_cast<size_t>(kRedBlocksMax) ? b : kRedBlocksMax);
}

template <typename T, typename TF>
void launch_energy_t(const void *I, const void *A, int W, int H, const void *F, const void *B,
                     int fw, int fh, int w, int h, float omega, float eps, const int *stop,
                     double *part, int nb, hipStream_t s) {
    hipLaunchKernelGGL((energy_partial_kernel<T, TF>), dim3(nb), dim3(kRedThreads), 0, s,
                       static_cast<const T *>(I), static_cast<const T *>(A), W, H,
                       static_cast<const TF *>(F), static_cast<const TF *>(B), fw, fh, w, h, omega,
                       eps, stop, part);
}

int launch_energy(const void *I, const void *A, int W, int H, const void *F, const void *B, int w,
                  int h, float omega, float eps, int storage, int state_storage, const int *stop,
                  double *part, double *out, void *stream) {
    return launch_energy_mapped(I, A, W, H, F, B, w, h, w, h, omega, eps, storage, state_storage,
                                stop, part, out, stream);
}

// The partial sums of launch_energy_mapped (one launch).
int launch_energy_parts(const void *I, const void *A, int W, int H, const void *F, const void *B,
                        int fw, int fh, int w, int h, float omega, float eps, int storage,
                        int state_storage, const int *stop, double *part, hipStream_t s) {
    const int nb = energy_blocks(w, h);
    const bool i16 = storage == FGE_F16, f16 = state_storage == FGE_F16;
    if (i16 && f16)
        launch_energy_t<_Float16, _Float16>(I, A, W, H, F, B, fw, fh, w, h, omega, eps, stop, part, nb, s);
    else if (i16)
        launch_energy_t<_Float16, float>(I, A, W, H, F, B, fw, fh, w, h, omega, eps, stop, part, nb, s);
    else if (f16)
        launch_energy_t<float, _Float16>(I, A, W, H, F, B, fw, fh, w, h, omega, eps, stop, part, nb, s);
    else
        launch_energy_t<float, float>(I, A, W, H, F, B, fw, fh, w, h, omega, eps, stop, part, nb, s);
    return static_cast<int>(hipGetLastError());
}

int launch_energy_mapped(const void *I, const void *A, int W, int H, const void *F, const void *B,
                         int fw, int fh, int w, int h, float omega, float eps, int storage,
                         int state_storage, const int *stop, double *part, double *out,
                         void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int err = launch_energy_parts(I, A, W, H, F, B, fw, fh, w, h, omega, eps, storage,
                                        state_storage, stop, part, s);
    if (err) return err;
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kRedThreads), 0, s, part,
                       energy_blocks(w, h), stop, out);
    return static_cast<int>(hipGetLastError());
}

int launch_energy_check(const void *I, const void *A, int W, int H, const void *F, const void *B,
                        int w, int h, float omega, float eps, int storage, int state_storage,
                        double *part, double *out, double *eprev, int *stop, int *count,
                        double tol, int k, int kmax, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int err = launch_energy_parts(I, A, W, H, F, B, w, h, w, h, omega, eps, storage,
                                        state_storage, stop, part, s);
    if (err) return err;
    hipLaunchKernelGGL(energy_check_kernel, dim3(1), dim3(kRedThreads), 0, s, part,
                       energy_blocks(w, h), out, eprev, stop, count, tol, k, kmax);
    return static_cast<int>(hipGetLastError());
}

int launch_energy_final(const double *part, int nb, double *out, void *stream) {
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kRedThreads), 0,
                       static_cast<hipStream_t>(stream), part, nb, nullptr, out);
    return static_cast<int>(hipGetLastError());
}

int launch_pass_final(const double *part, int nb, double *out, PassCtl *ctl, int m, double tol,
                      long seq, void *stream) {
    hipLaunchKernelGGL(pass_final_kernel, dim3(1), dim3(kRedThreads), 0,
                       static_cast<hipStream_t>(stream), part, nb, out, ctl, m, tol,
                       static_cast<double>(seq));
    return static_cast<int>(hipGetLastError());
}

}  // namespace fge

extern "C" {

size_t fge_energy_workspace_bytes(int32_t H, int32_t W) {
    if (W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return 0;
    return (static_cast<size_t>(fge::energy_blocks(W, H)) * 5 * sizeof(double) + 255) & ~static_cast<size_t>(255);
}

fge_status fge_energy(const void *I, const void *alpha, const void *F, const void *B, int32_t H,
                      int32_t W, const fge_params *p, double *out, void *workspace,
                      size_t workspace_bytes, void *stream) {
    fge_params tmp;
    if (!p) {
        fge_default_params(&tmp);
        p = &tmp;
    }
    if (!fge::params_valid(*p)) return FGE_EINVAL;
    if (W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return FGE_EINVAL;
    if (!I || !alpha || !F || !B || !out) return FGE_EINVAL;
    const size_t need = fge_energy_workspace_bytes(H, W);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return FGE_EWORKSPACE;
    return fge::launch_energy(I, alpha, W, H, F, B, W, H, p->omega, p->eps_r, p->storage,
                              p->storage, nullptr, static_cast<double *>(workspace), out, stream)
               ? FGE_EHIP
               : FGE_OK;
}

size_t fge_quality_workspace_bytes(int32_t H, int32_t W) {
    if (W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return 0;
    const size_t tiles = static_cast<size_t>((W + fge::kQTx - 1) / fge::kQTx) * ((H + fge::kQTy - 1) / fge::kQTy);
    const size_t nb = std::max(tiles, static_cast<size_t>(fge::energy_blocks(W, H)));
    return (nb * 4 * sizeof(double) + 255) & ~static_cast<size_t>(255);
}

fge_status fge_quality(const void *F, const void *G, const void *alpha, int32_t H, int32_t W,
                       int32_t dtype, double sigma, double *out, void *workspace,
                       size_t workspace_bytes, void *stream) {
    if (!F || !G || !alpha || !out || W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide)
        return FGE_EINVAL;
    if (dtype != FGE_F32 && dtype != FGE_F16) return FGE_EINVAL;
    const int r = static_cast<int>(4.0 * sigma + 0.5);
    if (!(sigma > 0.0) || r < 1 || r > fge::kGradMaxR) return FGE_EINVAL;
    const size_t need = fge_quality_workspace_bytes(H, W);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return FGE_EWORKSPACE;
    fge::GradFilter K{};
    K.r = r;
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) sum += (K.phi[r + j] = std::exp(-0.5 * j * j / (sigma * sigma)));
    for (int j = -r; j <= r; ++j) {
        K.phi[r + j] /= sum;
        K.der[r + j] = j / (sigma * sigma) * K.phi[r + j];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(workspace);
    if (r <= fge::kQMaxR) {
        const dim3 grid((W + fge::kQTx - 1) / fge::kQTx, (H + fge::kQTy - 1) / fge::kQTy);
        if (dtype == FGE_F16)
            hipLaunchKernelGGL(fge::quality_tile_kernel<_Float16>, grid, dim3(fge::kQThreads), 0, s,
                               static_cast<const _Float16 *>(F), static_cast<const _Float16 *>(G),
                               static_cast<const _Float16 *>(alpha), W, H, K, part);
        else
            hipLaunchKernelGGL(fge::quality_tile_kernel<float>, grid, dim3(fge::kQThreads), 0, s,
                               static_cast<const float *>(F), static_cast<const float *>(G),
                               static_cast<const float *>(alpha), W, H, K, part);
        if (hipGetLastError() != hipSuccess) return FGE_EHIP;
        hipLaunchKernelGGL(fge::quality_final_kernel, dim3(1), dim3(fge::kRedThreads), 0, s, part,
                           static_cast<int>(grid.x * grid.y), out);
        return hipGetLastError() == hipSuccess ? FGE_OK : FGE_EHIP;
    }
    const int nb = fge::energy_blocks(W, H);
    if (dtype == FGE_F16)
        hipLaunchKernelGGL(fge::quality_partial_kernel<_Float16>, dim3(nb), dim3(fge::kRedThreads),
                           0, s, static_cast<const _Float16 *>(F), static_cast<const _Float16 *>(G),
                           static_cast<const _Float16 *>(alpha), W, H, K, part);
    else
        hipLaunchKernelGGL(fge::quality_partial_kernel<float>, dim3(nb), dim3(fge::kRedThreads), 0,
                           s, static_cast<const float *>(F), static_cast<const float *>(G),
                           static_cast<const float *>(alpha), W, H, K, part);
    if (hipGetLastError() != hipSuccess) return FGE_EHIP;
    hipLaunchKernelGGL(fge::quality_final_kernel, dim3(1), dim3(fge::kRedThreads), 0, s, part, nb, out);
    return hipGetLastError() == hipSuccess ? FGE_OK : FGE_EHIP;
}

fge_status fge_composite(const void *F, const void *alpha, const void *B, int32_t H, int32_t W,
                         int32_t dtype, void *C, void *stream) {
    if (!F || !alpha || !B || !C || W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide)
        return FGE_EINVAL;
    if (dtype != FGE_F32 && dtype != FGE_F16) return FGE_EINVAL;
    const size_t n = static_cast<size_t>(W) * H;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    if (dtype == FGE_F16)
        hipLaunchKernelGGL(fge::composite_kernel<_Float16>, grid, dim3(256), 0, s,
                           static_cast<const _Float16 *>(F), static_cast<const _Float16 *>(alpha),
                           static_cast<const _Float16 *>(B), static_cast<_Float16 *>(C), n);
    else
        hipLaunchKernelGGL(fge::composite_kernel<float>, grid, dim3(256), 0, s,
                           static_cast<const float *>(F), static_cast<const float *>(alpha),
                           static_cast<const float *>(B), static_cast<float *>(C), n);
    return hipGetLastError() == hipSuccess ? FGE_OK : FGE_EHIP;
}

fge_status fge_hwc_to_planar(const void *src, int32_t src_dtype, int32_t channels, int32_t H,
                             int32_t W, void *planes, void *alpha, int32_t dst_dtype,
                             void *stream) {
    if (!src || !planes || W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return FGE_EINVAL;
    if (channels != 3 && channels != 4) return FGE_EINVAL;
    if (channels == 4 && !alpha) return FGE_EINVAL;
    if (!fge::dtype_ok(src_dtype) || !fge::dtype_ok(dst_dtype)) return FGE_EINVAL;
    const size_t n = static_cast<size_t>(W) * H;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *al = channels == 4 ? alpha : nullptr;
    int err;
    switch (src_dtype) {
        case FGE_F32: err = fge::launch_h2p_src<float>(src, channels, n, dst_dtype, planes, al, s); break;
        case FGE_F16: err = fge::launch_h2p_src<_Float16>(src, channels, n, dst_dtype, planes, al, s); break;
        default: err = fge::launch_h2p_src<uint8_t>(src, channels, n, dst_dtype, planes, al, s); break;
    }
    return err ? FGE_EHIP : FGE_OK;
}

fge_status fge_planar_to_hwc(const void *planes, int32_t src_dtype, int32_t H, int32_t W,
                             void *dst, int32_t dst_dtype, void *stream) {
    if (!planes || !dst || W < 1 || H < 1 || W > fge::kMaxSide || H > fge::kMaxSide) return FGE_EINVAL;
    if (!fge::dtype_ok(src_dtype) || !fge::dtype_ok(dst_dtype)) return FGE_EINVAL;
    const size_t n = static_cast<size_t>(W) * H;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int err;
    switch (src_dtype) {
        case FGE_F32: err = fge::launch_p2h_src<float>(planes, n, dst_dtype, dst, s); break;
        case FGE_F16: err = fge::launch_p2h_src<_Float16>(planes, n, dst_dtype, dst, s); break;
        default: err = fge::launch_p2h_src<uint8_t>(planes, n, dst_dtype, dst, s); break;
    }
    return err ? FGE_EHIP : FGE_OK;
}

}  // extern "C"
