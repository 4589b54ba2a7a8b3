/* The C oracle's entry points on small images, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py: every order of the fixed-count
 * pipeline, the convergence form, the explicit sweep schedule, both smooth resizes and the
 * energy, over sizes from 1x1 to several levels with ragged edges.  The sanitizers abort on a
 * finding; the driver itself checks only that every value stays finite and in [0, 1]. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int fgo_num_levels(int w, int h);
int fgo_ml(const double *I, const double *a, int W, int H, double omega, double eps,
           int small_size, int iters_small, int iters_big, int order, const double *init_f,
           const double *init_b, double *F, double *B);
double fgo_energy(const double *F, const double *B, const double *I, const double *a, int w,
                  int h, double omega, double eps);
int fgo_ml_schedule(const double *I, const double *a, int W, int H, double omega, double eps,
                    int order, const int *sweeps, double *F, double *B);
int fgo_ml_converge(const double *I, const double *a, int W, int H, double omega, double eps,
                    int order, double tol, int max_sweeps, int *sweeps_out, double *F, double *B);
int fgo_ml_resize(const double *I, const double *a, int W, int H, double omega, double eps,
                  int order, int resize, const int *sweeps, double *F, double *B);

static unsigned rng = 7;
static double urand(void) {
    rng = rng * 1103515245u + 12345u;
    return (double)((rng >> 8) & 0xFFFF) / 65535.0;
}

static int check(const double *v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i]) || v[i] < 0.0 || v[i] > 1.0) return 0;
    return 1;
}

int main(void) {
    static const int sizes[][2] = {{1, 1}, {2, 1}, {1, 3}, {5, 4}, {17, 9}, {33, 31}, {70, 45}};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) {
        const int W = sizes[s][0], H = sizes[s][1];
        const size_t n = (size_t)W * H;
        double *I = malloc(3 * n * sizeof(double)), *a = malloc(n * sizeof(double));
        double *F = malloc(3 * n * sizeof(double)), *B = malloc(3 * n * sizeof(double));
        for (size_t i = 0; i < 3 * n; ++i) I[i] = urand();
        for (size_t i = 0; i < n; ++i) a[i] = urand();
        for (int order = 0; order < 3; ++order) {
            if (fgo_ml(I, a, W, H, 0.1, 5e-3, 32, 10, 2, order, NULL, NULL, F, B) < 1) return 1;
            if (!check(F, 3 * n) || !check(B, 3 * n)) return 1;
            if (!isfinite(fgo_energy(F, B, I, a, W, H, 0.1, 5e-3))) return 1;
            int sw[16];
            if (fgo_ml_converge(I, a, W, H, 0.1, 5e-3, order, 1e-4, 50, sw, F, B) < 1) return 1;
            if (fgo_ml_schedule(I, a, W, H, 0.1, 5e-3, order, sw, F, B) < 1) return 1;
            for (int resize = 0; resize < 2; ++resize)
                if (fgo_ml_resize(I, a, W, H, 0.1, 5e-3, order, resize, sw, F, B) < 1) return 1;
            if (!check(F, 3 * n) || !check(B, 3 * n)) return 1;
        }
        free(I);
        free(a);
        free(F);
        free(B);
    }
    printf("oracle: ok\n");
    return 0;
}
