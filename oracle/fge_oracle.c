/*
 * FP64 CPU oracle for multi-level foreground estimation
 * (Germer, Uelwer, Conrad, Harmeling: "Fast Multi-Level Foreground Estimation", arXiv 2006.14970).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU path is checked
 * against.  Only tests, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links, includes or calls anything here, and nothing here comes from the
 * product library.
 *
 * What it computes (all in IEEE double, no blocking, no fusion, no reordering):
 *   - Algorithm 1 (Section III-D, "Implementation"): the multi-level driver, with the level count
 *     n_l = ceil(log2(max(w, h))), level sizes round(w^(l/n_l)), round(h^(l/n_l)), a resize of the
 *     full-resolution image and matte and of the previous level's F and B to every level, and a
 *     fixed number of sweeps per level (10 when the level is at most 32x32, else 2; Section III-D
 *     text before Algorithm 1).
 *   - The per-pixel update: the 2x2 system of eq. 9 in its matrix form (data term of eq. 1 plus
 *     the neighbour sums with weights eps_r + omega |alpha_i - alpha_j| of eq. 3 over the four
 *     clamped neighbours), solved by Cramer's rule, then clamped to [0, 1].
 *   - The global quadratic energy whose stationarity conditions are the per-pixel equations.
 *
 * Readings where the paper is silent (each is listed with its reason in the design notes):
 *   - N_i is the 4-neighbourhood (left, right, up, down); out-of-range neighbours are clamped to
 *     the image, so a border pixel sees itself (Algorithm 1, neighbour clamp).
 *   - "resize" is nearest-neighbour with source index (x * w_src) / w_dst in integer arithmetic.
 *   - "low resolution" means w <= 32 and h <= 32.
 *   - A 1x1 input gets one level (the formula gives zero).
 *   - Sweep order: raster (the paper's sequential in-place loop, y outer, x inner), red-black
 *     (all pixels with (x + y) even, then all odd, each in place) or Jacobi (every pixel from the
 *     previous sweep's values).
 *
 * Built twice: plain (every loop on one thread) and with OpenMP, where the rows of one colour of a
 * red-black sweep, or the rows of a Jacobi sweep, are split over threads.  Every pixel's
 * arithmetic is the same in both builds, so their results are bit-identical.
 *
 * Layout: planar, row-major, x fastest.  A 3-channel image of size w x h is 3 planes of w*h
 * doubles (plane c starts at c*w*h); the matte is one plane.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { FGO_RASTER = 0, FGO_REDBLACK = 1, FGO_JACOBI = 2 };

/* Number of levels, Algorithm 1: ceil(log2(max(w, h))), at least 1. */
int fgo_num_levels(int w, int h)
{
    int m = w > h ? w : h;
    int n = 0;
    /* smallest n with 2^n >= m, computed with integers so no rounding enters */
    while (((long long)1 << n) < (long long)m) n++;
    return n < 1 ? 1 : n;
}

/* Level size, Algorithm 1: round(full^(level / num_levels)). */
int fgo_level_size(int full, int level, int num_levels)
{
    double v = pow((double)full, (double)level / (double)num_levels);
    return (int)floor(v + 0.5);
}

/* Nearest-neighbour resize of `planes` planes from ws x hs to wd x hd. */
void fgo_resize_nearest(const double *src, int ws, int hs, int planes, double *dst, int wd, int hd)
{
    for (int c = 0; c < planes; c++) {
        for (int y = 0; y < hd; y++) {
            int ys = (int)(((long long)y * hs) / hd);
            for (int x = 0; x < wd; x++) {
                int xs = (int)(((long long)x * ws) / wd);
                dst[(size_t)c * wd * hd + (size_t)y * wd + x] =
                    src[(size_t)c * ws * hs + (size_t)ys * ws + xs];
            }
        }
    }
}

static double clamp01(double v)
{
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

static int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/*
 * Solve the per-pixel system of eq. 9 for pixel (x, y), reading F and B from (Fs, Bs) and the
 * input I and matte a, and return the clamped solution in fout[3], bout[3].
 *
 * Eq. 9 in matrix form: with U = [a_i, 1 - a_i]^T, the weights s_j = eps + omega |a_i - a_j| of
 * the four clamped neighbours (eq. 3), S = sum_j s_j, P_c = sum_j s_j F_j^c and
 * Q_c = sum_j s_j B_j^c, the unknown g_c = (F_i^c, B_i^c) solves
 *     (U U^T + S Id) g_c = U I_i^c + (P_c, Q_c)^T,
 * the same 2x2 matrix for the three channels.  It is solved by Cramer's rule, and each component
 * is then clamped to [0, 1] (the clamp that follows the solve in Algorithm 1).
 */
static void solve_pixel(const double *Fs, const double *Bs, const double *I, const double *a,
                        int w, int h, int x, int y, double omega, double eps,
                        double fout[3], double bout[3])
{
    const size_t plane = (size_t)w * h;
    const size_t i = (size_t)y * w + x;
    const double u0 = a[i], u1 = 1.0 - a[i];

    /* neighbour sums: left, right, up, down, each coordinate clamped to the image */
    const int nx[4] = {clampi(x - 1, 0, w - 1), clampi(x + 1, 0, w - 1), x, x};
    const int ny[4] = {y, y, clampi(y - 1, 0, h - 1), clampi(y + 1, 0, h - 1)};
    double S = 0.0, P[3] = {0.0, 0.0, 0.0}, Q[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 4; k++) {
        const size_t j = (size_t)ny[k] * w + nx[k];
        const double s = eps + omega * fabs(u0 - a[j]);
        S += s;
        for (int c = 0; c < 3; c++) {
            P[c] += s * Fs[c * plane + j];
            Q[c] += s * Bs[c * plane + j];
        }
    }

    /* M = U U^T + S Id */
    const double m00 = u0 * u0 + S, m01 = u0 * u1, m11 = u1 * u1 + S;
    const double det = m00 * m11 - m01 * m01;
    for (int c = 0; c < 3; c++) {
        const double r0 = u0 * I[c * plane + i] + P[c];
        const double r1 = u1 * I[c * plane + i] + Q[c];
        fout[c] = clamp01((m11 * r0 - m01 * r1) / det);
        bout[c] = clamp01((m00 * r1 - m01 * r0) / det);
    }
}

static void update_in_place(double *F, double *B, const double *I, const double *a,
                            int w, int h, int x, int y, double omega, double eps)
{
    const size_t plane = (size_t)w * h;
    const size_t i = (size_t)y * w + x;
    double f[3], g[3];
    solve_pixel(F, B, I, a, w, h, x, y, omega, eps, f, g);
    for (int c = 0; c < 3; c++) {
        F[c * plane + i] = f[c];
        B[c * plane + i] = g[c];
    }
}

/* Threads a parallel region uses: 1 unless built with OpenMP. */
int fgo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One sweep over every pixel of a w x h level, in the given order, updating F and B. */
void fgo_sweep(double *F, double *B, const double *I, const double *a, int w, int h,
               double omega, double eps, int order)
{
    if (order == FGO_RASTER) {
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++)
                update_in_place(F, B, I, a, w, h, x, y, omega, eps);
    } else if (order == FGO_REDBLACK) {
        /* A pixel of one colour reads only pixels of the other colour (and, through the border
         * clamp, itself), so the rows of one colour may be split over threads (OpenMP build):
         * every pixel gets the same value in any split. */
        for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for schedule(static)
            for (int y = 0; y < h; y++)
                for (int x = 0; x < w; x++)
                    if (((x + y) & 1) == colour)
                        update_in_place(F, B, I, a, w, h, x, y, omega, eps);
        }
    } else {
        const size_t plane = (size_t)w * h;
        double *Fo = (double *)malloc(3 * plane * sizeof(double));
        double *Bo = (double *)malloc(3 * plane * sizeof(double));
        memcpy(Fo, F, 3 * plane * sizeof(double));
        memcpy(Bo, B, 3 * plane * sizeof(double));
#pragma omp parallel for schedule(static)
        for (int y = 0; y < h; y++) {
            for (int x = 0; x < w; x++) {
                double f[3], g[3];
                size_t i = (size_t)y * w + x;
                solve_pixel(Fo, Bo, I, a, w, h, x, y, omega, eps, f, g);
                for (int c = 0; c < 3; c++) {
                    F[c * plane + i] = f[c];
                    B[c * plane + i] = g[c];
                }
            }
        }
        free(Fo);
        free(Bo);
    }
}

/*
 * Algorithm 1.  I: 3 x H x W, a: H x W, outputs F, B: 3 x H x W each.
 * init_f / init_b: the three channel values of the 1x1 starting F and B (the paper uses zeros;
 * NULL means zeros).  Returns the number of levels run.
 */
int fgo_ml(const double *I, const double *a, int W, int H, double omega, double eps,
           int small_size, int iters_small, int iters_big, int order,
           const double *init_f, const double *init_b, double *F, double *B)
{
    const int n = fgo_num_levels(W, H);
    int wp = 1, hp = 1;
    double *Fp = (double *)calloc(3, sizeof(double));
    double *Bp = (double *)calloc(3, sizeof(double));
    for (int c = 0; c < 3; c++) {
        Fp[c] = init_f ? init_f[c] : 0.0;
        Bp[c] = init_b ? init_b[c] : 0.0;
    }

    for (int l = 1; l <= n; l++) {
        int w = fgo_level_size(W, l, n);
        int h = fgo_level_size(H, l, n);
        size_t plane = (size_t)w * h;
        double *Il = (double *)malloc(3 * plane * sizeof(double));
        double *al = (double *)malloc(plane * sizeof(double));
        double *Fl = (double *)malloc(3 * plane * sizeof(double));
        double *Bl = (double *)malloc(3 * plane * sizeof(double));

        fgo_resize_nearest(I, W, H, 3, Il, w, h);
        fgo_resize_nearest(a, W, H, 1, al, w, h);
        fgo_resize_nearest(Fp, wp, hp, 3, Fl, w, h);
        fgo_resize_nearest(Bp, wp, hp, 3, Bl, w, h);

        int iters = (w <= small_size && h <= small_size) ? iters_small : iters_big;
        for (int it = 0; it < iters; it++)
            fgo_sweep(Fl, Bl, Il, al, w, h, omega, eps, order);

        free(Il);
        free(al);
        free(Fp);
        free(Bp);
        Fp = Fl;
        Bp = Bl;
        wp = w;
        hp = h;
    }

    /* the last level has the full size, since round(W^1) = W */
    memcpy(F, Fp, 3 * (size_t)W * H * sizeof(double));
    memcpy(B, Bp, 3 * (size_t)W * H * sizeof(double));
    free(Fp);
    free(Bp);
    return n;
}

/*
 * Quadratic energy whose stationary point every sweep order approaches while no clamp is active:
 *   E = sum_i sum_c (a_i F_i^c + (1 - a_i) B_i^c - I_i^c)^2
 *     + sum over undirected in-image 4-neighbour edges {i, j} of
 *       (eps + omega |a_i - a_j|) sum_c [(F_i^c - F_j^c)^2 + (B_i^c - B_j^c)^2].
 * Setting dE/dF_i, dE/dB_i to zero gives, pixel by pixel, the normal equations of eq. 9 (the
 * weights are symmetric in i and j, so every edge is counted once).
 */
double fgo_energy(const double *F, const double *B, const double *I, const double *a,
                  int w, int h, double omega, double eps)
{
    const size_t plane = (size_t)w * h;
    double e = 0.0;
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            size_t i = (size_t)y * w + x;
            for (int c = 0; c < 3; c++) {
                double r = a[i] * F[c * plane + i] + (1.0 - a[i]) * B[c * plane + i] - I[c * plane + i];
                e += r * r;
            }
            /* right and down edges, so each edge appears once */
            for (int k = 0; k < 2; k++) {
                int xj = x + (k == 0), yj = y + (k == 1);
                if (xj >= w || yj >= h) continue;
                size_t j = (size_t)yj * w + xj;
                double s = eps + omega * fabs(a[i] - a[j]);
                for (int c = 0; c < 3; c++) {
                    double df = F[c * plane + i] - F[c * plane + j];
                    double db = B[c * plane + i] - B[c * plane + j];
                    e += s * (df * df + db * db);
                }
            }
        }
    }
    return e;
}

/*
 * Algorithm 1 with a given number of sweeps per level: level l runs sweeps[l-1] sweeps (fgo_ml's
 * fixed rule is the schedule 10 / 2).  Replays a schedule decided elsewhere.  Returns the number
 * of levels.
 */
int fgo_ml_schedule(const double *I, const double *a, int W, int H, double omega, double eps,
                    int order, const int *sweeps, double *F, double *B)
{
    const int n = fgo_num_levels(W, H);
    int wp = 1, hp = 1;
    double *Fp = (double *)calloc(3, sizeof(double));
    double *Bp = (double *)calloc(3, sizeof(double));
    for (int l = 1; l <= n; l++) {
        int w = fgo_level_size(W, l, n);
        int h = fgo_level_size(H, l, n);
        size_t plane = (size_t)w * h;
        double *Il = (double *)malloc(3 * plane * sizeof(double));
        double *al = (double *)malloc(plane * sizeof(double));
        double *Fl = (double *)malloc(3 * plane * sizeof(double));
        double *Bl = (double *)malloc(3 * plane * sizeof(double));
        fgo_resize_nearest(I, W, H, 3, Il, w, h);
        fgo_resize_nearest(a, W, H, 1, al, w, h);
        fgo_resize_nearest(Fp, wp, hp, 3, Fl, w, h);
        fgo_resize_nearest(Bp, wp, hp, 3, Bl, w, h);
        for (int it = 0; it < sweeps[l - 1]; it++)
            fgo_sweep(Fl, Bl, Il, al, w, h, omega, eps, order);
        free(Il);
        free(al);
        free(Fp);
        free(Bp);
        Fp = Fl;
        Bp = Bl;
        wp = w;
        hp = h;
    }
    memcpy(F, Fp, 3 * (size_t)W * H * sizeof(double));
    memcpy(B, Bp, 3 * (size_t)W * H * sizeof(double));
    free(Fp);
    free(Bp);
    return n;
}

/*
 * Algorithm 1's "while not converged" form, the test taken every m sweeps: at every level, after
 * the resize, run m sweeps at a time until the level's energy (fgo_energy of the level's F, B
 * against its resized image and matte) changes over those m sweeps by at most tol times its value
 * before them, or until max_checks groups have run; at least one group runs.  E before the first
 * group is the energy of the resized start.  checks_out[l-1] receives the groups level l ran.
 * When rel_out is not NULL, rel_out[(l-1) * rel_cap + k] receives |E_k - E_(k+1)| / E_k of the
 * (k+1)-th group of level l, for k < rel_cap (the quantity the stopping test compares with tol).
 * Returns the number of levels.
 */
int fgo_ml_converge_every(const double *I, const double *a, int W, int H, double omega, double eps,
                          int order, int m, double tol, int max_checks, int *checks_out,
                          double *rel_out, int rel_cap, double *F, double *B)
{
    const int n = fgo_num_levels(W, H);
    int wp = 1, hp = 1;
    double *Fp = (double *)calloc(3, sizeof(double));
    double *Bp = (double *)calloc(3, sizeof(double));
    for (int l = 1; l <= n; l++) {
        int w = fgo_level_size(W, l, n);
        int h = fgo_level_size(H, l, n);
        size_t plane = (size_t)w * h;
        double *Il = (double *)malloc(3 * plane * sizeof(double));
        double *al = (double *)malloc(plane * sizeof(double));
        double *Fl = (double *)malloc(3 * plane * sizeof(double));
        double *Bl = (double *)malloc(3 * plane * sizeof(double));
        fgo_resize_nearest(I, W, H, 3, Il, w, h);
        fgo_resize_nearest(a, W, H, 1, al, w, h);
        fgo_resize_nearest(Fp, wp, hp, 3, Fl, w, h);
        fgo_resize_nearest(Bp, wp, hp, 3, Bl, w, h);
        double e_prev = fgo_energy(Fl, Bl, Il, al, w, h, omega, eps);
        int k = 0;
        for (;;) {
            for (int s = 0; s < m; s++)
                fgo_sweep(Fl, Bl, Il, al, w, h, omega, eps, order);
            double e = fgo_energy(Fl, Bl, Il, al, w, h, omega, eps);
            double rel = fabs(e_prev - e) / e_prev;
            if (rel_out && k < rel_cap)
                rel_out[(size_t)(l - 1) * rel_cap + k] = rel;
            k++;
            if (fabs(e_prev - e) <= tol * e_prev || k >= max_checks) break;
            e_prev = e;
        }
        checks_out[l - 1] = k;
        free(Il);
        free(al);
        free(Fp);
        free(Bp);
        Fp = Fl;
        Bp = Bl;
        wp = w;
        hp = h;
    }
    memcpy(F, Fp, 3 * (size_t)W * H * sizeof(double));
    memcpy(B, Bp, 3 * (size_t)W * H * sizeof(double));
    free(Fp);
    free(Bp);
    return n;
}

/* The test after every sweep (m = 1): sweeps_out[l-1] receives the sweeps level l ran. */
int fgo_ml_converge(const double *I, const double *a, int W, int H, double omega, double eps,
                    int order, double tol, int max_sweeps, int *sweeps_out, double *F, double *B)
{
    return fgo_ml_converge_every(I, a, W, H, omega, eps, order, 1, tol, max_sweeps, sweeps_out,
                                 NULL, 0, F, B);
}

/*
 * The smooth resize variant (the paper leaves the resize kernel open).
 *
 * Area resize: destination pixel (x, y) is the mean of the source over its footprint
 * [x ws/wd, (x+1) ws/wd) x [y hs/hd, (y+1) hs/hd), every source pixel weighted by its overlap
 * with it.  The weights are separable: the 1-D overlap of source index i with destination
 * interval [x0, x1) is max(0, min(i + 1, x1) - max(i, x0)), divided by the interval length.
 */
static void area_weights(int ns, int nd, int x, int *lo, int *hi, double *w)
{
    double x0 = (double)x * ns / nd, x1 = (double)(x + 1) * ns / nd;
    int i0 = (int)floor(x0), i1 = (int)ceil(x1);
    if (i1 > ns) i1 = ns;
    *lo = i0;
    *hi = i1;
    for (int i = i0; i < i1; i++) {
        double a = i > x0 ? i : x0, b = i + 1 < x1 ? i + 1 : x1;
        w[i - i0] = (b - a) / (x1 - x0);
    }
}

void fgo_resize_area(const double *src, int ws, int hs, int planes, double *dst, int wd, int hd)
{
    double *wx = (double *)malloc(((size_t)ws + 2) * sizeof(double));
    double *wy = (double *)malloc(((size_t)hs + 2) * sizeof(double));
    for (int c = 0; c < planes; c++) {
        for (int y = 0; y < hd; y++) {
            int ylo, yhi;
            area_weights(hs, hd, y, &ylo, &yhi, wy);
            for (int x = 0; x < wd; x++) {
                int xlo, xhi;
                area_weights(ws, wd, x, &xlo, &xhi, wx);
                double acc = 0.0;
                for (int j = ylo; j < yhi; j++)
                    for (int i = xlo; i < xhi; i++)
                        acc += wy[j - ylo] * wx[i - xlo] * src[(size_t)c * ws * hs + (size_t)j * ws + i];
                dst[(size_t)c * wd * hd + (size_t)y * wd + x] = acc;
            }
        }
    }
    free(wx);
    free(wy);
}

/*
 * Bilinear resize with pixel centres at half-integers: the destination pixel x samples source
 * coordinate u = (x + 1/2) ws/wd - 1/2, clamped to [0, ws - 1]; it mixes source pixels floor(u)
 * and floor(u) + 1 (clamped) with weights 1 - (u - floor(u)) and u - floor(u); likewise in y.
 */
static void bilinear_tap(int ns, int nd, int x, int *i0, int *i1, double *f)
{
    double u = ((double)x + 0.5) * ns / nd - 0.5;
    if (u < 0.0) u = 0.0;
    if (u > ns - 1) u = ns - 1;
    *i0 = (int)floor(u);
    *i1 = *i0 + 1 < ns ? *i0 + 1 : ns - 1;
    *f = u - *i0;
}

void fgo_resize_bilinear(const double *src, int ws, int hs, int planes, double *dst, int wd, int hd)
{
    for (int c = 0; c < planes; c++) {
        const double *s = src + (size_t)c * ws * hs;
        for (int y = 0; y < hd; y++) {
            int y0, y1;
            double fy;
            bilinear_tap(hs, hd, y, &y0, &y1, &fy);
            for (int x = 0; x < wd; x++) {
                int x0, x1;
                double fx;
                bilinear_tap(ws, wd, x, &x0, &x1, &fx);
                double top = (1.0 - fx) * s[(size_t)y0 * ws + x0] + fx * s[(size_t)y0 * ws + x1];
                double bot = (1.0 - fx) * s[(size_t)y1 * ws + x0] + fx * s[(size_t)y1 * ws + x1];
                dst[(size_t)c * wd * hd + (size_t)y * wd + x] = (1.0 - fy) * top + fy * bot;
            }
        }
    }
}

/*
 * Algorithm 1 with the resize variant `resize` (0: nearest, as fgo_ml; 1: smooth -- area for the
 * full-resolution image and matte, bilinear for the previous level's F and B) and sweeps[l-1]
 * sweeps at level l.
 */
int fgo_ml_resize(const double *I, const double *a, int W, int H, double omega, double eps,
                  int order, int resize, const int *sweeps, double *F, double *B)
{
    const int n = fgo_num_levels(W, H);
    int wp = 1, hp = 1;
    double *Fp = (double *)calloc(3, sizeof(double));
    double *Bp = (double *)calloc(3, sizeof(double));
    for (int l = 1; l <= n; l++) {
        int w = fgo_level_size(W, l, n);
        int h = fgo_level_size(H, l, n);
        size_t plane = (size_t)w * h;
        double *Il = (double *)malloc(3 * plane * sizeof(double));
        double *al = (double *)malloc(plane * sizeof(double));
        double *Fl = (double *)malloc(3 * plane * sizeof(double));
        double *Bl = (double *)malloc(3 * plane * sizeof(double));
        if (resize == 1) {
            fgo_resize_area(I, W, H, 3, Il, w, h);
            fgo_resize_area(a, W, H, 1, al, w, h);
            fgo_resize_bilinear(Fp, wp, hp, 3, Fl, w, h);
            fgo_resize_bilinear(Bp, wp, hp, 3, Bl, w, h);
        } else {
            fgo_resize_nearest(I, W, H, 3, Il, w, h);
            fgo_resize_nearest(a, W, H, 1, al, w, h);
            fgo_resize_nearest(Fp, wp, hp, 3, Fl, w, h);
            fgo_resize_nearest(Bp, wp, hp, 3, Bl, w, h);
        }
        for (int it = 0; it < sweeps[l - 1]; it++)
            fgo_sweep(Fl, Bl, Il, al, w, h, omega, eps, order);
        free(Il);
        free(al);
        free(Fp);
        free(Bp);
        Fp = Fl;
        Bp = Bl;
        wp = w;
        hp = h;
    }
    memcpy(F, Fp, 3 * (size_t)W * H * sizeof(double));
    memcpy(B, Bp, 3 * (size_t)W * H * sizeof(double));
    free(Fp);
    free(Bp);
    return n;
}
