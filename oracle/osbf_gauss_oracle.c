/*
 * One-sided Gaussian filter (Sec. II-B, separable kernels) -- CPU FP64
 * oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never calls it and shares no code, header or constant with it.
 *
 * Every window sum is taken directly over its pixel set, in double precision.
 *
 * Conventions (readings of the paper):
 *  - The 1D kernel is the Gaussian g(u) = exp(-u^2 / (2 sigma^2)) on
 *    |u| <= r.  Its one-sided parts are normalised separately (the
 *    normalisation of the one-sided kernels in Sec. II-B); the full kernel is
 *    normalised over [-r, r].  As for the box filter, both one-sided parts
 *    contain the centre tap (reading of the centre-inclusion question).
 *  - The eight windows, their pixel sets and their order (= tie order) are
 *    those of the box filter: R, L, D, U, SE, SW, NE, NW; a window's weight
 *    at offset (a, b) from the pixel is g(a) g(b), and its mean is the
 *    weighted sum divided by the sum of its weights.  sigma = +infinity gives
 *    the one-sided box filter.
 *  - Selection: the first window whose mean is closest to the pixel value
 *    (Alg. 2 with these kernels); the new value is that mean.  T Jacobi
 *    sweeps; every sweep reads the replicate extension of the iterate.
 *  - A window's weight total is the product of its two 1D totals, Zh =
 *    sum_{u=0..r} g(u) for a one-sided axis and Zf = sum_{u=-r..r} g(u) for a
 *    full one, so mirror-image windows share one normaliser and exact ties
 *    stay exact.
 *  - err reports N |mean_i - c| with N = Zh^2 Zf, the scale the GPU kernel
 *    compares in.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int clampg(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Pixel offsets of window w: a in [ax0, ax1], b in [by0, by1]. */
static void gauss_window(int w, int r, int *ax0, int *ax1, int *by0, int *by1)
{
    /* R L D U SE SW NE NW */
    static const int xs[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    static const int ys[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    *ax0 = xs[w] > 0 ? 0 : -r;
    *ax1 = xs[w] < 0 ? 0 : r;
    *by0 = ys[w] > 0 ? 0 : -r;
    *by1 = ys[w] < 0 ? 0 : r;
}

static double gauss_tap(int u, double sigma)
{
    if (isinf(sigma)) return 1.0;
    return exp(-(double)u * u / (2.0 * sigma * sigma));
}

/*
 * One Jacobi sweep on one plane.
 *   sel  nullable [H][W]; err nullable [H][W][8] (N |mean_i - c|);
 *   mean nullable [H][W][8]
 */
void oracle_gauss_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean,
                        int H, int W, int r, double sigma, int nthreads)
{
    double zh = 0.0, zf = 0.0;
    for (int t = 0; t <= r; ++t) zh += gauss_tap(t, sigma);
    for (int t = -r; t <= r; ++t) zf += gauss_tap(t, sigma);
    const double N = zh * zh * zf;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            const double c = u[p];
            int m = 0;
            double best = 0.0, mbest = 0.0;
            for (int w = 0; w < 8; ++w) {
                int ax0, ax1, by0, by1;
                gauss_window(w, r, &ax0, &ax1, &by0, &by1);
                double s = 0.0;
                for (int b = by0; b <= by1; ++b)
                    for (int a = ax0; a <= ax1; ++a)
                        s += gauss_tap(a, sigma) * gauss_tap(b, sigma) *
                             u[(size_t)clampg(y + b, 0, H - 1) * W + clampg(x + a, 0, W - 1)];
                const double z = (ax1 - ax0 == r ? zh : zf) * (by1 - by0 == r ? zh : zf);
                const double mu = s / z;
                const double e = fabs(mu - c);
                if (err) err[p * 8 + w] = N * e;
                if (mean) mean[p * 8 + w] = mu;
                if (w == 0 || e < best) { best = e; m = w; mbest = mu; }
            }
            out[p] = mbest;
            if (sel) sel[p] = (uint8_t)m;
        }
    }
    (void)nthreads;
}

/* T sweeps on `planes` planes; in and out may alias; sel nullable [T][planes][H][W]. */
int oracle_gauss_forward(const double *in, double *out, uint8_t *sel, int planes, int H, int W, int r,
                         double sigma, int T, int nthreads)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0 || !(sigma > 0.0)) return -1;
    const size_t n = (size_t)H * W;
    if (n == 0 || planes == 0) return 0;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int pl = 0; pl < planes; ++pl) {
        memcpy(a, in + (size_t)pl * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            oracle_gauss_sweep(a, b, sel ? sel + ((size_t)t * planes + pl) * n : NULL, NULL, NULL, H, W,
                               r, sigma, nthreads);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(out + (size_t)pl * n, a, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}
