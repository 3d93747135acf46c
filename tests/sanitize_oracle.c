/* Driver for the sanitizer build of the C oracle (test infrastructure): every
 * entry point of oracle/*.c on shapes where windows reach far past the image
 * (1x1, 1xN, Nx1, r larger than the image) and on ordinary ragged shapes.
 * Built with -fsanitize=address,undefined by tests/test_oracle_sanitize.py,
 * which fails on any sanitizer report or a non-zero exit. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_forward(const double *in, double *out, uint8_t *sel, int planes, int H, int W, int r, int T,
                   int nthreads);
int oracle_forward_padonce(const double *in, double *out, int planes, int H, int W, int r, int T);
void oracle_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean, int H, int W, int r,
                  int nthreads);
void oracle_select_int64(const int64_t *in, uint8_t *sel, int64_t *sums, int H, int W, int r);
void oracle_apply_fixed(const double *x, const uint8_t *sel, double *y, int H, int W, int r);
void oracle_adjoint_scatter(const double *g_next, const uint8_t *sel, double *g, int H, int W, int r);
int oracle_backward(const double *in, const double *grad_out, double *grad_in, uint8_t *sel_out, int planes,
                    int H, int W, int r, int T, int nthreads);
void oracle_fast_sweep(const double *u, double *out, uint8_t *sel, double *cand, int H, int W, int r,
                       int nthreads);
int oracle_fast_forward(const double *in, double *out, int planes, int H, int W, int r, int T, int nthreads);
int oracle_box_forward(const double *in, double *out, int planes, int H, int W, int r, int T);
void oracle_gauss_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean, int H, int W,
                        int r, double sigma, int nthreads);
int oracle_gauss_forward(const double *in, double *out, uint8_t *sel, int planes, int H, int W, int r,
                         double sigma, int T, int nthreads);
void oracle3d_sweep(const double *u, double *out, uint8_t *sel, double *err, double *mean, int D, int H,
                    int W, int r, int nthreads);
int oracle3d_forward(const double *in, double *out, uint8_t *sel, int vols, int D, int H, int W, int r,
                     int T, int nthreads);
void oracle3d_select_int64(const int64_t *u, uint8_t *sel, int64_t *sums, int D, int H, int W, int r);

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

#define ALLOC(T, n) ((T *)malloc(sizeof(T) * (size_t)(n) + 1))

static int planar(int P, int H, int W, int r, int T) {
    const size_t n = (size_t)P * H * W, hw = (size_t)H * W;
    double *in = ALLOC(double, n), *out = ALLOC(double, n), *g = ALLOC(double, n), *gi = ALLOC(double, n);
    double *err = ALLOC(double, hw * 8), *mean = ALLOC(double, hw * 8), *cand = ALLOC(double, hw * 8);
    uint8_t *sel = ALLOC(uint8_t, n * (T > 0 ? T : 1)), *s1 = ALLOC(uint8_t, hw);
    int64_t *iu = ALLOC(int64_t, hw), *sums = ALLOC(int64_t, hw * 8);
    for (size_t i = 0; i < n; ++i) { in[i] = urand(); g[i] = urand() - 0.5; }
    for (size_t i = 0; i < hw; ++i) iu[i] = (int64_t)(urand() * 256);
    int bad = 0;
    bad |= oracle_forward(in, out, sel, P, H, W, r, T, 1);
    bad |= oracle_forward_padonce(in, out, P, H, W, r, T);
    oracle_sweep(in, out, s1, err, mean, H, W, r, 1);
    oracle_select_int64(iu, s1, sums, H, W, r);
    oracle_apply_fixed(in, s1, out, H, W, r);
    oracle_adjoint_scatter(g, s1, gi, H, W, r);
    bad |= oracle_backward(in, g, gi, sel, P, H, W, r, T, 1);
    oracle_fast_sweep(in, out, s1, cand, H, W, r, 1);
    bad |= oracle_fast_forward(in, out, P, H, W, r, T, 1);
    bad |= oracle_box_forward(in, out, P, H, W, r, T);
    if (r <= 8) {
        oracle_gauss_sweep(in, out, s1, err, mean, H, W, r, 0.5 * r + 0.3, 1);
        bad |= oracle_gauss_forward(in, out, sel, P, H, W, r, 0.5 * r + 0.3, T, 1);
    }
    free(in); free(out); free(g); free(gi); free(err); free(mean); free(cand); free(sel); free(s1);
    free(iu); free(sums);
    return bad;
}

static int volume(int V, int D, int H, int W, int r, int T) {
    const size_t n = (size_t)V * D * H * W, dhw = (size_t)D * H * W;
    double *in = ALLOC(double, n), *out = ALLOC(double, n);
    double *err = ALLOC(double, dhw * 14), *mean = ALLOC(double, dhw * 14);
    uint8_t *sel = ALLOC(uint8_t, n * (T > 0 ? T : 1)), *s1 = ALLOC(uint8_t, dhw);
    int64_t *iu = ALLOC(int64_t, dhw), *sums = ALLOC(int64_t, dhw * 14);
    for (size_t i = 0; i < n; ++i) in[i] = urand();
    for (size_t i = 0; i < dhw; ++i) iu[i] = (int64_t)(urand() * 256);
    int bad = oracle3d_forward(in, out, sel, V, D, H, W, r, T, 1);
    oracle3d_sweep(in, out, s1, err, mean, D, H, W, r, 1);
    oracle3d_select_int64(iu, s1, sums, D, H, W, r);
    free(in); free(out); free(err); free(mean); free(sel); free(s1); free(iu); free(sums);
    return bad;
}

int main(void) {
    static const int shapes[][3] = {{1, 1, 1}, {1, 1, 17}, {1, 17, 1}, {2, 3, 2}, {1, 23, 29}, {3, 9, 40}};
    static const int radii[] = {0, 1, 2, 3, 5, 16, 32};
    int bad = 0;
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (size_t k = 0; k < sizeof radii / sizeof radii[0]; ++k)
            bad |= planar(shapes[s][0], shapes[s][1], shapes[s][2], radii[k], 2);
    static const int vshapes[][4] = {{1, 1, 1, 1}, {1, 1, 5, 7}, {2, 4, 3, 6}, {1, 9, 8, 7}};
    for (size_t s = 0; s < sizeof vshapes / sizeof vshapes[0]; ++s)
        for (int r = 0; r <= 4; ++r)
            bad |= volume(vshapes[s][0], vshapes[s][1], vshapes[s][2], vshapes[s][3], r, 2);
    printf("sanitize_oracle: %s\n", bad ? "entry point returned an error" : "ok");
    return bad ? 1 : 0;
}
