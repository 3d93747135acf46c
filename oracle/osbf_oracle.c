/*
 * One-sided box filter -- CPU FP64 oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never calls it and shares no code, header or constant with it.
 *
 * Everything here is deliberately plain and slow: every window sum is taken
 * directly over its pixel set, pixel by pixel, in double precision.
 *
 * Conventions (readings of the paper, each stated once):
 *  - A plane is H rows by W columns, row-major; x is the column index
 *    (growing rightwards), y is the row index (growing downwards).
 *  - Windows (Sec. II-A, Eq. 6-13; box kernels of Sec. III-A): every window
 *    contains the centre pixel.  With y pointing down the paper's sets map as
 *      N1 = SW, N2 = SE, N3 = NE, N4 = NW, N5 = L, N6 = R, N7 = D, N8 = U.
 *    Quadrants hold (r+1)^2 pixels, halves (r+1)(2r+1) pixels.
 *  - Tie order (first minimum wins): R, L, D, U, SE, SW, NE, NW.  This is the
 *    order of the eight difference planes in the appendix listing once the
 *    documented 'same' convolution is applied to its one-sided kernels.
 *  - Distance: Alg. 2 takes argmin |k_i (x) U - U|.  Multiplying every
 *    distance by N = (r+1)^2 (2r+1) does not change the argmin, so the oracle
 *    compares e_i = |w_i S_i - N c| with w = 2r+1 for quadrants and r+1 for
 *    halves (S_i the window sum, c the centre value).  On integer-valued
 *    inputs every e_i is an exact integer in double precision, so exact ties
 *    are resolved exactly by the stated order.
 *  - Update: the new value is the selected mean S_m / n_m (equal to
 *    U + d_m of Alg. 2 in exact arithmetic).
 *  - Iterations: exactly T Jacobi sweeps (every pixel of sweep t+1 reads
 *    sweep t only); T = 0 is the identity.  Alg. 2's loop bound reads as
 *    T+1 sweeps, the appendix loop as T; T is taken.
 *  - Boundary, default ("clamp") mode: every sweep reads the replicate
 *    extension of the current iterate, P(x,y) = U(clamp(x), clamp(y)).
 *    The "pad-once" mode instead follows the appendix: replicate-pad once by
 *    r, evolve the whole padded frame with zero extension beyond it (the
 *    divisor stays n_i), crop at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O_R = 0, O_L, O_D, O_U, O_SE, O_SW, O_NE, O_NW, O_NWIN };

int oracle_version(void) { return 3; }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Pixel set of window w at (x,y): [x0,x1] x [y0,y1] (Eq. 6-13). */
void oracle_window_extent(int w, int x, int y, int r, int *x0, int *x1, int *y0, int *y1)
{
    switch (w) {
    case O_R:  *x0 = x;     *x1 = x + r; *y0 = y - r; *y1 = y + r; break;
    case O_L:  *x0 = x - r; *x1 = x;     *y0 = y - r; *y1 = y + r; break;
    case O_D:  *x0 = x - r; *x1 = x + r; *y0 = y;     *y1 = y + r; break;
    case O_U:  *x0 = x - r; *x1 = x + r; *y0 = y - r; *y1 = y;     break;
    case O_SE: *x0 = x;     *x1 = x + r; *y0 = y;     *y1 = y + r; break;
    case O_SW: *x0 = x - r; *x1 = x;     *y0 = y;     *y1 = y + r; break;
    case O_NE: *x0 = x;     *x1 = x + r; *y0 = y - r; *y1 = y;     break;
    default:   *x0 = x - r; *x1 = x;     *y0 = y - r; *y1 = y;     break;
    }
}

/* Number of pixels of window w (box kernels of Sec. III-A). */
static double window_count(int w, int r)
{
    return (w >= O_SE) ? (double)(r + 1) * (r + 1) : (double)(r + 1) * (2 * r + 1);
}

/* Weight that turns a window sum into N times its mean. */
static double window_scale(int w, int r)
{
    return (w >= O_SE) ? (double)(2 * r + 1) : (double)(r + 1);
}

/* Direct sum of window w at (x,y) over the replicate extension of u. */
static double window_sum_clamp(const double *u, int H, int W, int w, int x, int y, int r)
{
    int x0, x1, y0, y1;
    oracle_window_extent(w, x, y, r, &x0, &x1, &y0, &y1);
    double s = 0.0;
    for (int yy = y0; yy <= y1; ++yy)
        for (int xx = x0; xx <= x1; ++xx)
            s += u[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)];
    return s;
}

/* Direct sum of window w at (x,y) with zero extension outside [0,H)x[0,W). */
static double window_sum_zero(const double *u, int H, int W, int w, int x, int y, int r)
{
    int x0, x1, y0, y1;
    oracle_window_extent(w, x, y, r, &x0, &x1, &y0, &y1);
    double s = 0.0;
    for (int yy = y0; yy <= y1; ++yy)
        for (int xx = x0; xx <= x1; ++xx)
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) s += u[(size_t)yy * W + xx];
    return s;
}

/* Selection of Alg. 2 at one pixel, given the eight window sums. */
static int select_window(const double S[O_NWIN], double c, int r, double *e_out)
{
    const double N = (double)(r + 1) * (r + 1) * (2 * r + 1);
    int m = 0;
    double best = 0.0;
    for (int i = 0; i < O_NWIN; ++i) {
        double e = fabs(window_scale(i, r) * S[i] - N * c);
        if (e_out) e_out[i] = e;
        if (i == 0 || e < best) { best = e; m = i; }
    }
    return m;
}

/*
 * One Jacobi sweep of Alg. 2 on one plane, clamp boundary.
 *   u    [H][W]        current iterate (read only)
 *   out  [H][W]        next iterate (must not alias u)
 *   sel  [H][W]        nullable; selected window index 0..7
 *   err  [H][W][8]     nullable; e_i = |w_i S_i - N c| for every window
 *   mean [H][W][8]     nullable; S_i / n_i for every window
 */
void oracle_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean,
                  int H, int W, int r, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double S[O_NWIN];
            for (int i = 0; i < O_NWIN; ++i) S[i] = window_sum_clamp(u, H, W, i, x, y, r);
            size_t p = (size_t)y * W + x;
            int m = select_window(S, u[p], r, err ? err + p * O_NWIN : NULL);
            out[p] = S[m] / window_count(m, r);
            if (sel) sel[p] = (uint8_t)m;
            if (mean)
                for (int i = 0; i < O_NWIN; ++i) mean[p * O_NWIN + i] = S[i] / window_count(i, r);
        }
    }
    (void)nthreads;
}

/*
 * T sweeps of Alg. 2 (clamp boundary) on `planes` independent planes.
 *   in, out   [planes][H][W]   may alias
 *   sel       nullable [T][planes][H][W]
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_forward(const double *in, double *out, uint8_t *sel,
                   int planes, int H, int W, int r, int T, int nthreads)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    size_t n = (size_t)H * W;
    if (n == 0 || planes == 0) return 0;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int pl = 0; pl < planes; ++pl) {
        memcpy(a, in + (size_t)pl * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            uint8_t *s = sel ? sel + ((size_t)t * planes + pl) * n : NULL;
            oracle_sweep(a, b, s, NULL, NULL, H, W, r, nthreads);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(out + (size_t)pl * n, a, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}

/*
 * Pad-once ("appendix") reading: replicate-pad each plane once by r, run T
 * sweeps on the padded frame where pixels beyond the frame count as zero and
 * every divisor stays n_i, then crop the frame back to H x W.
 */
int oracle_forward_padonce(const double *in, double *out, int planes, int H, int W,
                           int r, int T)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    int Hp = H + 2 * r, Wp = W + 2 * r;
    size_t np = (size_t)Hp * Wp;
    if ((size_t)H * W == 0 || planes == 0) return 0;
    double *a = (double *)malloc(np * sizeof(double));
    double *b = (double *)malloc(np * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int pl = 0; pl < planes; ++pl) {
        const double *src = in + (size_t)pl * H * W;
        for (int y = 0; y < Hp; ++y)
            for (int x = 0; x < Wp; ++x)
                a[(size_t)y * Wp + x] = src[(size_t)clampi(y - r, 0, H - 1) * W + clampi(x - r, 0, W - 1)];
        for (int t = 0; t < T; ++t) {
            for (int y = 0; y < Hp; ++y)
                for (int x = 0; x < Wp; ++x) {
                    double S[O_NWIN];
                    for (int i = 0; i < O_NWIN; ++i) S[i] = window_sum_zero(a, Hp, Wp, i, x, y, r);
                    size_t p = (size_t)y * Wp + x;
                    int m = select_window(S, a[p], r, NULL);
                    b[p] = S[m] / window_count(m, r);
                }
            double *tmp = a; a = b; b = tmp;
        }
        double *dst = out + (size_t)pl * H * W;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                dst[(size_t)y * W + x] = a[(size_t)(y + r) * Wp + (x + r)];
    }
    free(a); free(b);
    return 0;
}

/*
 * Exact selection for integer-valued input, one sweep: window sums and the
 * scaled distances |w_i S_i - N c| are computed in int64, so ties are exact.
 *   in  [H][W] int64, sel [H][W], sums nullable [H][W][8]
 */
void oracle_select_int64(const int64_t *in, uint8_t *sel, int64_t *sums, int H, int W, int r)
{
    const int64_t N = (int64_t)(r + 1) * (r + 1) * (2 * r + 1);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int m = 0;
            int64_t best = 0;
            for (int i = 0; i < O_NWIN; ++i) {
                int x0, x1, y0, y1;
                oracle_window_extent(i, x, y, r, &x0, &x1, &y0, &y1);
                int64_t s = 0;
                for (int yy = y0; yy <= y1; ++yy)
                    for (int xx = x0; xx <= x1; ++xx)
                        s += in[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)];
                if (sums) sums[((size_t)y * W + x) * O_NWIN + i] = s;
                int64_t w = (i >= O_SE) ? (2 * r + 1) : (r + 1);
                int64_t e = w * s - N * in[(size_t)y * W + x];
                if (e < 0) e = -e;
                if (i == 0 || e < best) { best = e; m = i; }
            }
            sel[(size_t)y * W + x] = (uint8_t)m;
        }
}

/*
 * The sweep as a linear map with its selection held fixed:
 *   y(p) = (1/n_m) * sum over q in window m(p) of x(clamp(q)).
 */
void oracle_apply_fixed(const double *x, const uint8_t *sel, double *y, int H, int W, int r)
{
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            size_t p = (size_t)py * W + px;
            int m = sel[p];
            y[p] = window_sum_clamp(x, H, W, m, px, py, r) / window_count(m, r);
        }
}

/*
 * Adjoint of oracle_apply_fixed, written as the plain scatter: every pixel p
 * spreads g_next(p)/n_m(p) over the clamped pixels of its selected window.
 *   g [H][W] is overwritten.
 */
void oracle_adjoint_scatter(const double *g_next, const uint8_t *sel, double *g,
                            int H, int W, int r)
{
    memset(g, 0, (size_t)H * W * sizeof(double));
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            size_t p = (size_t)py * W + px;
            int m = sel[p];
            double v = g_next[p] / window_count(m, r);
            int x0, x1, y0, y1;
            oracle_window_extent(m, px, py, r, &x0, &x1, &y0, &y1);
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx)
                    g[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)] += v;
        }
}

/*
 * Gradient of the T-sweep filter (clamp mode) with every selection held at
 * its forward value: grad_in = A_0^T A_1^T ... A_{T-1}^T grad_out.
 *   in, grad_out, grad_in [planes][H][W]; sel_out nullable [T][planes][H][W].
 */
int oracle_backward(const double *in, const double *grad_out, double *grad_in,
                    uint8_t *sel_out, int planes, int H, int W, int r, int T, int nthreads)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    size_t n = (size_t)H * W;
    if (n == 0 || planes == 0) return 0;
    uint8_t *sel = (uint8_t *)malloc((size_t)(T > 0 ? T : 1) * n);
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!sel || !a || !b) { free(sel); free(a); free(b); return -1; }
    for (int pl = 0; pl < planes; ++pl) {
        memcpy(a, in + (size_t)pl * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            oracle_sweep(a, b, sel + (size_t)t * n, NULL, NULL, H, W, r, nthreads);
            if (sel_out) memcpy(sel_out + ((size_t)t * planes + pl) * n, sel + (size_t)t * n, n);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(a, grad_out + (size_t)pl * n, n * sizeof(double));
        for (int t = T - 1; t >= 0; --t) {
            oracle_adjoint_scatter(a, sel + (size_t)t * n, b, H, W, r);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(grad_in + (size_t)pl * n, a, n * sizeof(double));
    }
    free(sel); free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------
 * Fast approximation (Alg. 3, Sec. III-F).
 *
 * Readings: the one field computed per sweep is the mean of the north-west
 * ("left up", y pointing down) quadrant ending at the pixel,
 *   Qm(x,y) = mean of P over [x-r, x] x [y-r, y];
 * the four quadrant candidates are its shifts by {0, r} in x and y
 * (NW = Qm(x,y), NE = Qm(x+r,y), SW = Qm(x,y+r), SE = Qm(x+r,y+r)), and each
 * half window is replaced by the average of its two quadrants (eq:app):
 *   R ~ (NE+SE)/2, L ~ (NW+SW)/2, D ~ (SW+SE)/2, U ~ (NW+NE)/2.
 * The new value is the candidate closest to the current one, ties in the
 * order R, L, D, U, SE, SW, NE, NW (as for the exact filter); the printed
 * update U + d(x+u,y+v) is read as "take the selected candidate".
 * ------------------------------------------------------------------------ */

/* Mean of P over [x-r, x] x [y-r, y] with clamped coordinates. */
static double nw_mean_clamp(const double *u, int H, int W, int x, int y, int r)
{
    double s = 0.0;
    for (int yy = y - r; yy <= y; ++yy)
        for (int xx = x - r; xx <= x; ++xx)
            s += u[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)];
    return s / ((double)(r + 1) * (r + 1));
}

/* One sweep of the fast approximation; cand nullable [H][W][8]. */
void oracle_fast_sweep(const double *u, double *out, uint8_t *sel, double *cand,
                       int H, int W, int r, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const double nw = nw_mean_clamp(u, H, W, x, y, r);
            const double ne = nw_mean_clamp(u, H, W, x + r, y, r);
            const double sw = nw_mean_clamp(u, H, W, x, y + r, r);
            const double se = nw_mean_clamp(u, H, W, x + r, y + r, r);
            double a[O_NWIN];
            a[O_R] = 0.5 * (ne + se);
            a[O_L] = 0.5 * (nw + sw);
            a[O_D] = 0.5 * (sw + se);
            a[O_U] = 0.5 * (nw + ne);
            a[O_SE] = se;
            a[O_SW] = sw;
            a[O_NE] = ne;
            a[O_NW] = nw;
            const size_t p = (size_t)y * W + x;
            const double c = u[p];
            int m = 0;
            double best = 0.0;
            for (int i = 0; i < O_NWIN; ++i) {
                const double e = fabs(a[i] - c);
                if (i == 0 || e < best) { best = e; m = i; }
                if (cand) cand[p * O_NWIN + i] = a[i];
            }
            out[p] = a[m];
            if (sel) sel[p] = (uint8_t)m;
        }
    }
    (void)nthreads;
}

/* T sweeps of the fast approximation on `planes` planes (clamp boundary). */
int oracle_fast_forward(const double *in, double *out, int planes, int H, int W, int r, int T,
                        int nthreads)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    size_t n = (size_t)H * W;
    if (n == 0 || planes == 0) return 0;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int pl = 0; pl < planes; ++pl) {
        memcpy(a, in + (size_t)pl * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            oracle_fast_sweep(a, b, NULL, NULL, H, W, r, nthreads);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(out + (size_t)pl * n, a, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------
 * Classical box filter (the paper's timing baseline, Table I): the mean of
 * P over the full window [x-r, x+r] x [y-r, y+r], clamp boundary, T sweeps.
 * ------------------------------------------------------------------------ */
int oracle_box_forward(const double *in, double *out, int planes, int H, int W, int r, int T)
{
    if (planes < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    size_t n = (size_t)H * W;
    if (n == 0 || planes == 0) return 0;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    const double cnt = (double)(2 * r + 1) * (2 * r + 1);
    for (int pl = 0; pl < planes; ++pl) {
        memcpy(a, in + (size_t)pl * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    double s = 0.0;
                    for (int yy = y - r; yy <= y + r; ++yy)
                        for (int xx = x - r; xx <= x + r; ++xx)
                            s += a[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)];
                    b[(size_t)y * W + x] = s / cnt;
                }
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(out + (size_t)pl * n, a, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}
