// One-sided Gaussian filter (Sec. II-B separable kernels), gfx950.
//
// The box filter's eight windows, weighted by g(a) g(b) at offset (a, b) with
// g(u) = exp(-u^2 / (2 sigma^2)), g(0) = 1.  Because the weights separate,
// every window sum comes from one-sided 1D sums (O(r) per pixel):
//   Bm(x,y) = sum_{a=0..r} g(a) P(x-a, y),  Bp(x,y) = sum_{a=0..r} g(a) P(x+a, y)
//   NW = sum_b g(b) Bm(x, y-b), NE = sum_b g(b) Bp(x, y-b),
//   SW = sum_b g(b) Bm(x, y+b), SE = sum_b g(b) Bp(x, y+b),
//   Am = sum_b g(b) P(x, y-b),  Ap = sum_b g(b) P(x, y+b)        (b = 0..r)
//   R = NE + SE - Bp(x,y), L = NW + SW - Bm(x,y),
//   D = SW + SE - Ap,      U = NW + NE - Am
// (a full-range sum is the two one-sided sums minus the shared centre tap).
// Window means are S / (Zh Zh) for quadrants and S / (Zh Zf) for halves with
// Zh = sum_{u=0..r} g(u), Zf = 2 Zh - 1; distances are compared scaled by
// N = Zh^2 Zf (weight Zf for quadrants, Zh for halves) and the tournament of
// the box filter picks the first minimum.  sigma = infinity is the box filter.
//
// A workgroup (512 threads) owns a (64-2r)^2 tile and a 64 x 64 LDS region.
// Phase A computes Bm, Bp on the tile's columns over (row, r-column block)
// items; phase B gives each lane one output column, reads a block's 3r rows of
// Bm, Bp and P into registers, forms the window sums, selects and stores
// (coalesced along x).  Every sum adds its taps in the same order (centre
// first, then increasing distance) on both sides, so mirror-image windows of
// mirror-image data get identical bits.
#include "osbf_device.h"
#include "osbf_fwd_device.h"
#include "osbf_internal.h"

namespace osbf {

template <int R, bool SEL>
__global__ __launch_bounds__(512) void gauss_kernel(GaussLaunch a) {
    constexpr int NT = 512, RW = 64, RH = 64, PITCH = RW + 1, ARR = RH * PITCH, NY = NT / RW;
    extern __shared__ float lds[];
    float *const P = lds;
    float *const Bm = lds + ARR;
    float *const Bp = lds + 2 * ARR;
    const int tid = threadIdx.x, lx = tid % RW;
    const int ly = __builtin_amdgcn_readfirstlane(tid / RW);
    const int H = a.H, W = a.W, TW = a.tw, TH = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int t = xcd_remap(blockIdx.x, ntiles * a.planes);
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int X0 = (tile % a.tiles_x) * TW, Y0 = (tile / a.tiles_x) * TH;
    const int ox = X0 - R, oy = Y0 - R;
    const int xa = X0, xb = min(W, X0 + TW), ya = Y0, yb = min(H, Y0 + TH);
    const size_t plane_off = (size_t)plane * H * W;
    const float *src = a.src + plane_off;
    float g[R + 1];
#pragma unroll
    for (int i = 0; i <= R; ++i) g[i] = a.g[i];

    // clamped load of tile + halo, every row load issued before the first wait
    const int ry0 = max(0, oy), ry1 = min(H, Y0 + TH + R);
    {
        constexpr int NL = RH / NY;
        const int x = ox + lx;
        if (x >= 0 && x < W) {
            float raw[NL];
#pragma unroll
            for (int i = 0; i < NL; ++i) raw[i] = src[(size_t)min(ry0 + ly + i * NY, ry1 - 1) * W + x];
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int y = ry0 + ly + i * NY;
                if (y < ry1) P[(y - oy) * PITCH + lx] = raw[i];
            }
        }
    }
    __syncthreads();

    // Phase A: Bm, Bp on columns [xa, xb), rows [ry0, ry1); item = (row,
    // block of R columns), rows fastest.
    {
        const int nr = ry1 - ry0, nb = (xb - xa + R - 1) / R;
        const int lo = max(0, xa - R), hi = min(W, xb + R) - 1;  // columns in LDS
        const int dr = NT % nr, db = NT / nr;
        int b = tid / nr, row = tid - b * nr;
        while (b < nb) {
            const int rb = (ry0 + row - oy) * PITCH - ox;  // + image column
            const int x0 = xa + b * R;
            float p[3 * R];
#pragma unroll
            for (int i = 0; i < 3 * R; ++i) p[i] = P[rb + min(max(x0 - R + i, lo), hi)];
#pragma unroll
            for (int tt = 0; tt < R; ++tt) {
                if (x0 + tt < xb) {
                    float m = p[R + tt], q = p[R + tt];
#pragma unroll
                    for (int k = 1; k <= R; ++k) {
                        m = fmaf(g[k], p[R + tt - k], m);
                        q = fmaf(g[k], p[R + tt + k], q);
                    }
                    Bm[rb + x0 + tt] = m;
                    Bp[rb + x0 + tt] = q;
                }
            }
            row += dr;
            b += db;
            if (row >= nr) {
                row -= nr;
                ++b;
            }
        }
    }
    __syncthreads();

    // Phase B: lane = output column, blocks of R rows over the waves.
    const int x = ox + lx;
    if (x < xa || x >= xb) return;
    uint8_t *sel = SEL ? a.sel + plane_off : nullptr;
    float *dst = a.dst + plane_off;
    const float wq = a.w_q, wh = a.w_h, N = a.N, invN = a.invN;
    const int nblk = (yb - ya + R - 1) / R;
    for (int blk = ly; blk < nblk; blk += NY) {
        const int y0 = ya + blk * R;
        float vm[3 * R], vp[3 * R], vc[3 * R];
#pragma unroll
        for (int i = 0; i < 3 * R; ++i) {  // rows y0-R .. y0+2R-1, clamped
            const int yy = min(min(max(y0 - R + i, 0), H - 1), ry1 - 1);
            const int o = (yy - oy) * PITCH + lx;
            vm[i] = Bm[o];
            vp[i] = Bp[o];
            vc[i] = P[o];
        }
#pragma unroll
        for (int tt = 0; tt < R; ++tt) {
            const int y = y0 + tt;
            if (y >= yb) break;
            const int i = R + tt;
            float nw = vm[i], ne = vp[i], sw = vm[i], se = vp[i], am = vc[i], ap = vc[i];
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                nw = fmaf(g[k], vm[i - k], nw);
                ne = fmaf(g[k], vp[i - k], ne);
                sw = fmaf(g[k], vm[i + k], sw);
                se = fmaf(g[k], vp[i + k], se);
                am = fmaf(g[k], vc[i - k], am);
                ap = fmaf(g[k], vc[i + k], ap);
            }
            const float c = vc[i];
            const float nc = -N * c;
            float d[8];
            d[0] = fmaf(wh, ne + se - vp[i], nc);
            d[1] = fmaf(wh, nw + sw - vm[i], nc);
            d[2] = fmaf(wh, sw + se - ap, nc);
            d[3] = fmaf(wh, nw + ne - am, nc);
            d[4] = fmaf(wq, se, nc);
            d[5] = fmaf(wq, sw, nc);
            d[6] = fmaf(wq, ne, nc);
            d[7] = fmaf(wq, nw, nc);
            const Pick pk = select8<SEL>(d);
            const size_t gi = (size_t)y * W + x;
            dst[gi] = fmaf(pk.d, invN, c);
            if (SEL) sel[gi] = (uint8_t)pk.idx;
        }
    }
}

bool gauss_radius(int r) { return r >= 1 && r <= OSBF_GAUSS_MAX_R; }

void gauss_tile(int r, int *tw, int *th) { *tw = *th = 64 - 2 * r; }

template <int R>
static hipError_t launch_g(const GaussLaunch &a, hipStream_t stream) {
    constexpr size_t lds = (size_t)3 * 64 * 65 * sizeof(float);
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    if (a.sel)
        hipLaunchKernelGGL((gauss_kernel<R, true>), dim3(blocks), dim3(512), lds, stream, a);
    else
        hipLaunchKernelGGL((gauss_kernel<R, false>), dim3(blocks), dim3(512), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_gauss(const GaussLaunch &a, hipStream_t stream) {
    switch (a.r) {
        case 1: return launch_g<1>(a, stream);
        case 2: return launch_g<2>(a, stream);
        case 3: return launch_g<3>(a, stream);
        case 4: return launch_g<4>(a, stream);
        case 5: return launch_g<5>(a, stream);
        case 6: return launch_g<6>(a, stream);
        case 7: return launch_g<7>(a, stream);
        case 8: return launch_g<8>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace osbf
