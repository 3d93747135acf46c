/*
 * One-sided box filter on volumes (Sec. "Higher Dimension Case") -- CPU FP64
 * oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never calls it and shares no code, header or constant with it.
 *
 * Every window sum is taken directly over its voxel set, voxel by voxel, in
 * double precision.
 *
 * Conventions (readings of the paper, each stated once):
 *  - A volume is D slices of H rows by W columns, slice-major then row-major;
 *    x is the column, y the row, z the slice index.
 *  - Windows: the one-sided kernels k^- / k^+ and the full kernel k along
 *    each axis span 6 half windows (one axis one-sided, the other two full)
 *    and 8 octants (one-sided along all three axes).  Every window contains
 *    the centre voxel.  Halves hold (r+1)(2r+1)^2 voxels, octants (r+1)^3.
 *  - Index (= tie order, first minimum wins), extending the planar order
 *    R, L, D, U, SE, SW, NE, NW (halves first, + side before - side, x before
 *    y, then octants with x varying fastest):
 *      0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z,
 *      6 (+x,+y,+z), 7 (-x,+y,+z), 8 (+x,-y,+z), 9 (-x,-y,+z),
 *     10 (+x,+y,-z), 11 (-x,+y,-z), 12 (+x,-y,-z), 13 (-x,-y,-z).
 *    The paper names the six halves but gives no order; this one is a reading.
 *  - Distance: argmin |mean_i - c| as in Alg. 2, compared as
 *    e_i = |w_i S_i - N c| with N = (r+1)^3 (2r+1)^2, w = (r+1)^2 for halves
 *    and (2r+1)^2 for octants; exact on integer-valued inputs.
 *  - Update: the selected mean S_m / n_m.  T Jacobi sweeps; T = 0 is the
 *    identity.  Every sweep reads the replicate extension of the current
 *    iterate (clamp in x, y and z).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O3_NWIN 14

static int clamp3(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Voxel set of window w at (x,y,z): [e0,e1] x [e2,e3] x [e4,e5]. */
void oracle3d_window_extent(int w, int x, int y, int z, int r, int *e)
{
    int c[3] = {x, y, z};
    /* side[a]: +1 one-sided towards +, -1 towards -, 0 full */
    int side[3] = {0, 0, 0};
    if (w < 6) {
        side[w / 2] = (w % 2 == 0) ? 1 : -1;
    } else {
        int o = w - 6;
        side[0] = (o & 1) ? -1 : 1;
        side[1] = (o & 2) ? -1 : 1;
        side[2] = (o & 4) ? -1 : 1;
    }
    for (int a = 0; a < 3; ++a) {
        e[2 * a] = side[a] > 0 ? c[a] : c[a] - r;
        e[2 * a + 1] = side[a] < 0 ? c[a] : c[a] + r;
    }
}

static double count3(int w, int r)
{
    return w < 6 ? (double)(r + 1) * (2 * r + 1) * (2 * r + 1) : (double)(r + 1) * (r + 1) * (r + 1);
}

static double scale3(int w, int r)
{
    return w < 6 ? (double)(r + 1) * (r + 1) : (double)(2 * r + 1) * (2 * r + 1);
}

static double window_sum3(const double *u, int D, int H, int W, int w, int x, int y, int z, int r)
{
    int e[6];
    oracle3d_window_extent(w, x, y, z, r, e);
    double s = 0.0;
    for (int zz = e[4]; zz <= e[5]; ++zz)
        for (int yy = e[2]; yy <= e[3]; ++yy)
            for (int xx = e[0]; xx <= e[1]; ++xx)
                s += u[((size_t)clamp3(zz, 0, D - 1) * H + clamp3(yy, 0, H - 1)) * W + clamp3(xx, 0, W - 1)];
    return s;
}

/*
 * One Jacobi sweep on one volume (clamp boundary).
 *   u    [D][H][W]       current iterate (read only)
 *   out  [D][H][W]       next iterate (must not alias u)
 *   sel  nullable [D][H][W]      selected window 0..13
 *   err  nullable [D][H][W][14]  e_i = |w_i S_i - N c|
 *   mean nullable [D][H][W][14]  S_i / n_i
 */
void oracle3d_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean,
                    int D, int H, int W, int r, int nthreads)
{
    const double N = (double)(r + 1) * (r + 1) * (r + 1) * (2 * r + 1) * (2 * r + 1);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
#endif
    for (int z = 0; z < D; ++z) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                const size_t p = ((size_t)z * H + y) * W + x;
                const double c = u[p];
                double S[O3_NWIN];
                int m = 0;
                double best = 0.0;
                for (int i = 0; i < O3_NWIN; ++i) {
                    S[i] = window_sum3(u, D, H, W, i, x, y, z, r);
                    const double e = fabs(scale3(i, r) * S[i] - N * c);
                    if (err) err[p * O3_NWIN + i] = e;
                    if (mean) mean[p * O3_NWIN + i] = S[i] / count3(i, r);
                    if (i == 0 || e < best) { best = e; m = i; }
                }
                out[p] = S[m] / count3(m, r);
                if (sel) sel[p] = (uint8_t)m;
            }
        }
    }
    (void)nthreads;
}

/*
 * T sweeps on `vols` independent volumes.
 *   in, out  [vols][D][H][W]   may alias
 *   sel      nullable [T][vols][D][H][W]
 */
int oracle3d_forward(const double *in, double *out, uint8_t *sel, int vols, int D, int H, int W,
                     int r, int T, int nthreads)
{
    if (vols < 0 || D < 0 || H < 0 || W < 0 || r < 0 || T < 0) return -1;
    const size_t n = (size_t)D * H * W;
    if (n == 0 || vols == 0) return 0;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int v = 0; v < vols; ++v) {
        memcpy(a, in + (size_t)v * n, n * sizeof(double));
        for (int t = 0; t < T; ++t) {
            uint8_t *s = sel ? sel + ((size_t)t * vols + v) * n : NULL;
            oracle3d_sweep(a, b, s, NULL, NULL, D, H, W, r, nthreads);
            double *tmp = a; a = b; b = tmp;
        }
        memcpy(out + (size_t)v * n, a, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}

/*
 * Exact integer selection for one sweep on an integer-valued volume: window
 * sums in int64 and e_i = |w_i S_i - N c| compared as integers.
 *   sums nullable [D][H][W][14]
 */
void oracle3d_select_int64(const int64_t *u, uint8_t *sel, int64_t *sums, int D, int H, int W, int r)
{
    const int64_t N = (int64_t)(r + 1) * (r + 1) * (r + 1) * (2 * r + 1) * (2 * r + 1);
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const size_t p = ((size_t)z * H + y) * W + x;
                int m = 0;
                int64_t best = 0;
                for (int i = 0; i < O3_NWIN; ++i) {
                    int e[6];
                    oracle3d_window_extent(i, x, y, z, r, e);
                    int64_t s = 0;
                    for (int zz = e[4]; zz <= e[5]; ++zz)
                        for (int yy = e[2]; yy <= e[3]; ++yy)
                            for (int xx = e[0]; xx <= e[1]; ++xx)
                                s += u[((size_t)clamp3(zz, 0, D - 1) * H + clamp3(yy, 0, H - 1)) * W +
                                       clamp3(xx, 0, W - 1)];
                    if (sums) sums[p * O3_NWIN + i] = s;
                    const int64_t w = i < 6 ? (int64_t)(r + 1) * (r + 1) : (int64_t)(2 * r + 1) * (2 * r + 1);
                    int64_t d = w * s - N * u[p];
                    if (d < 0) d = -d;
                    if (i == 0 || d < best) { best = d; m = i; }
                }
                sel[p] = (uint8_t)m;
            }
}
