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
// Two kernels compute the same sums in the same order (identical bits):
//
// * row streaming (the default): a workgroup of RW lanes owns a strip of
//   RW - 2r output columns (lane = strip column, halo of r on each side) and
//   a chunk of rows, and walks down it CH rows per step.  Only P passes
//   through LDS (a row sum needs the lane's neighbours); every lane keeps its
//   own column of Bm, Bp and P over the rows y-r .. y+r in registers, as a
//   ring of CH + 2r rows, so the vertical sums read no LDS at all.
// * tiled: a workgroup (512 threads) owns a (64-2r)^2 tile and a 64 x 64 LDS
//   region.  Phase A computes Bm, Bp on the tile's columns over (row,
//   r-column block) items; phase B gives each lane one output column, reads a
//   block's 3r rows of Bm, Bp and P into registers, forms the window sums,
//   selects and stores (coalesced along x).
//
// Every sum adds its taps in the same order (centre first, then increasing
// distance) on both sides, so mirror-image windows of mirror-image data get
// identical bits.
#include "osbf_device.h"
#include "osbf_fwd_device.h"
#include "osbf_internal.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace osbf {

// One-sided row sums at a staged row position p (p[-R..R] valid):
// m = sum_a g(a) P(x-a), q = sum_a g(a) P(x+a).
template <int R>
__device__ __forceinline__ void gauss_rowsums(const float *p, const float (&g)[R + 1], float &m, float &q) {
    m = p[0];
    q = p[0];
    static_for<1, R + 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        m = fmaf(g[k], p[-k], m);
        q = fmaf(g[k], p[k], q);
    });
}

// One output pixel from a lane's column window of Bm, Bp and P held in
// registers: row y + k (k in [-R, R]) sits at slot (I + k) mod L.  Forms the
// six one-sided column sums, the eight scaled distances and the tournament.
template <int R, int L, int I, bool SEL>
__device__ __forceinline__ Pick gauss_pixel(const float (&vm)[L], const float (&vp)[L], const float (&vc)[L],
                                            const float (&g)[R + 1], float wq, float wh, float N) {
    constexpr int c0 = I % L;
    float nw = vm[c0], ne = vp[c0], sw = vm[c0], se = vp[c0], am = vc[c0], ap = vc[c0];
    static_for<1, R + 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        constexpr int up = ((I - k) % L + L) % L, dn = (I + k) % L;
        nw = fmaf(g[k], vm[up], nw);
        ne = fmaf(g[k], vp[up], ne);
        sw = fmaf(g[k], vm[dn], sw);
        se = fmaf(g[k], vp[dn], se);
        am = fmaf(g[k], vc[up], am);
        ap = fmaf(g[k], vc[dn], ap);
    });
    const float nc = -N * vc[c0];
    float d[8];
    d[0] = fmaf(wh, ne + se - vp[c0], nc);
    d[1] = fmaf(wh, nw + sw - vm[c0], nc);
    d[2] = fmaf(wh, sw + se - ap, nc);
    d[3] = fmaf(wh, nw + ne - am, nc);
    d[4] = fmaf(wq, se, nc);
    d[5] = fmaf(wq, sw, nc);
    d[6] = fmaf(wq, ne, nc);
    d[7] = fmaf(wq, nw, nc);
    return select8<SEL>(d);
}

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
            static_for<0, R>([&](auto tv) {
                constexpr int tt = decltype(tv)::value;
                if (x0 + tt < xb) {
                    float m, q;
                    gauss_rowsums<R>(p + R + tt, g, m, q);
                    Bm[rb + x0 + tt] = m;
                    Bp[rb + x0 + tt] = q;
                }
            });
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
        static_for<0, R>([&](auto tv) {
            constexpr int tt = decltype(tv)::value;
            const int y = y0 + tt;
            if (y < yb) {
                const Pick pk = gauss_pixel<R, 3 * R, R + tt, SEL>(vm, vp, vc, g, wq, wh, N);
                const size_t gi = (size_t)y * W + x;
                dst[gi] = fmaf(pk.d, invN, vc[R + tt]);
                if (SEL) sel[gi] = (uint8_t)pk.idx;
            }
        });
    }
}

// ---------------------------------------------------------------------------
// Row-streaming kernel.  Ring row rho (rho >= 0) is image row Y0 - R + rho,
// clamped to the image, and sits in register slot rho mod L (L = CH + 2R).
// Step j loads ring rows j CH .. j CH + CH - 1 and, for each new row i,
// forms its row sums and then outputs image row Y0 + j CH - 2R + i, whose
// column window (ring rows j CH + i - 2R .. j CH + i) is then complete; the
// first 2R rows of a chunk only fill the ring.  The step body is unrolled over
// the ring's period so that every slot index is a constant.
constexpr int gauss_gcd(int a, int b) { return b == 0 ? a : gauss_gcd(b, a % b); }

// rows per step (the step body is unrolled (CH + 2R) / gcd(CH, 2R) times)
constexpr int gauss_step_rows(int r) { return r <= 2 ? 8 : r == 3 ? 6 : r == 5 ? 10 : r == 6 ? 6 : r == 7 ? 7 : 8; }

// Staging layout: column-major, a column's CH rows at an odd stride S, so a
// lane's 2R + 1 neighbours over all CH rows sit within the LDS instructions'
// immediate offsets of one base and lanes (stride S) hit distinct banks.
constexpr int gauss_col_stride(int r) { return gauss_step_rows(r) % 2 ? gauss_step_rows(r) + 2 : gauss_step_rows(r) + 1; }

// LDS: two staging buffers of RW + 2R columns (the lane's column at R, pads
// for the halo lanes' neighbours).
size_t gauss_stream_lds_bytes(int RW, int r) {
    return (size_t)2 * (RW + 2 * r) * gauss_col_stride(r) * sizeof(float);
}

// waves per SIMD to keep resident (caps the register budget)
constexpr int gauss_min_waves(int r) { return r >= 6 ? 4 : r >= 5 ? 5 : r >= 4 ? 6 : r >= 3 ? 7 : 8; }

template <int R, int RW, int CH, bool SEL>
__global__ __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(gauss_min_waves(R))))
void gauss_stream_kernel(GaussLaunch a) {
    constexpr int L = CH + 2 * R, PER = L / gauss_gcd(L, CH), S = CH % 2 ? CH + 2 : CH + 1;
    constexpr int BUF = (RW + 2 * R) * S;
    static_assert(2 * R * S + CH - 1 < 256, "a step's reads must fit the LDS immediate offsets");
    extern __shared__ float lds[];                // [2][RW + 2R][S]
    const int lx = threadIdx.x, me = R + lx;      // lane's staging column
    const int H = a.H, W = a.W, TW = a.tw, TH = a.th;
    const int nt = a.tiles_x * a.tiles_y;
    const int t = xcd_remap(blockIdx.x, nt * a.planes);
    const int plane = t / nt, tile = t - plane * nt;
    const int strip = tile / a.tiles_y, chunk = tile - strip * a.tiles_y;  // a strip's chunks adjacent
    const int X0 = strip * TW, Y0 = chunk * TH;
    const int x = X0 - R + lx;
    const bool out_col = lx >= R && lx < R + TW && x < W;
    const int y_end = min(H, Y0 + TH);
    const int nsteps = (2 * R + y_end - Y0 + CH - 1) / CH;
    const size_t plane_off = (size_t)plane * H * W;
    const float *src = a.src + plane_off + min(max(x, 0), W - 1);
    const int xo = out_col ? x : 0;
    float *dst = a.dst + plane_off + xo;
    uint8_t *sel = SEL ? a.sel + plane_off + xo : nullptr;
    float g[R + 1];
#pragma unroll
    for (int i = 0; i <= R; ++i) g[i] = a.g[i];
    const float wq = a.w_q, wh = a.w_h, N = a.N, invN = a.invN;
    const int ybase = Y0 - R;
    auto load_row = [&](int rho) { return src[(size_t)min(max(ybase + rho, 0), H - 1) * W]; };

    float vm[L], vp[L], vc[L], pf[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) pf[i] = load_row(i);

    // Staging buffer j & 1 is written before step j's barrier and read after
    // it; the next write to it (step j + 2) comes after step j + 1's barrier,
    // which every wave reaches only once its step-j reads are done.
    int j = 0;
    bool more = nsteps > 0;
    while (more) {
        static_for<0, PER>([&](auto phv) {
            constexpr int ph = decltype(phv)::value;
            if (!more) return;
            float *buf = lds + (j & 1) * BUF;
            static_for<0, CH>([&](auto iv) {
                constexpr int i = decltype(iv)::value;
                buf[me * S + i] = pf[i];
                vc[(ph * CH + i) % L] = pf[i];
            });
            if (j + 1 < nsteps) {
#pragma unroll
                for (int i = 0; i < CH; ++i) pf[i] = load_row((j + 1) * CH + i);
            }
            __syncthreads();
            // Row i: its row sums complete the column window of output row
            // y0 + i.  One row at a time, with the next row's neighbours read
            // ahead, keeps the live registers to the ring and two rows of taps.
            const float *col = buf + (me - R) * S;
            const int y0 = Y0 + j * CH - 2 * R;
            float pa[2 * R + 1], pn[2 * R + 1];
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k) pa[k] = col[k * S];
            static_for<0, CH>([&](auto iv) {
                constexpr int i = decltype(iv)::value;
                if constexpr (i + 1 < CH) {
#pragma unroll
                    for (int k = 0; k <= 2 * R; ++k) pn[k] = col[k * S + i + 1];
                }
                constexpr int slot = (ph * CH + i) % L;
                gauss_rowsums<R>(pa + R, g, vm[slot], vp[slot]);
                const int y = y0 + i;
                if (y >= Y0 && y < y_end) {
                    constexpr int I = (ph * CH + i - R + L) % L;
                    const Pick pk = gauss_pixel<R, L, I, SEL>(vm, vp, vc, g, wq, wh, N);
                    if (out_col) {
                        dst[(size_t)y * W] = fmaf(pk.d, invN, vc[I]);
                        if (SEL) sel[(size_t)y * W] = (uint8_t)pk.idx;
                    }
                }
                if constexpr (i + 1 < CH) {
#pragma unroll
                    for (int k = 0; k <= 2 * R; ++k) pa[k] = pn[k];
                }
                __builtin_amdgcn_sched_barrier(0);
            });
            ++j;
            more = j < nsteps;
        });
    }
}

bool gauss_radius(int r) { return r >= 1 && r <= OSBF_GAUSS_MAX_R; }

void gauss_tile(int r, int *tw, int *th) { *tw = *th = 64 - 2 * r; }

// Strip lanes and rows per workgroup of the streaming kernel by radius
// (rows 0: the launch fills the device's workgroup slots once), the fastest
// measured on 3 x 2048 x 2048 FP32 images with sigma = r / 2.
static const int kGaussPlan[OSBF_GAUSS_MAX_R + 1][2] = {
    {128, 0}, {256, 32}, {128, 0}, {128, 0}, {256, 16}, {256, 32}, {256, 32}, {128, 0}, {256, 0}};

bool gauss_geometry(GaussLaunch &a) {
    // OSBF_GAUSS: "tiled", or "stream[,lanes[,rows]]" (lanes 128 or 256,
    // rows per workgroup; 0 = fill the device once)
    int lanes = kGaussPlan[a.r][0], rows = kGaussPlan[a.r][1];
    bool tiled = false;
    if (const char *env = getenv("OSBF_GAUSS")) {
        if (!strncmp(env, "tiled", 5)) {
            tiled = true;
        } else if (!strncmp(env, "stream", 6)) {
            int l = 0, h = 0;
            const int n = sscanf(env + 6, ",%d,%d", &l, &h);
            if (n >= 1 && (l == 128 || l == 256)) lanes = l;
            if (n >= 2 && h >= 0) rows = h;
        }
    }
    if (tiled) {
        a.lanes = 0;
        gauss_tile(a.r, &a.tw, &a.th);
        a.tiles_x = (a.W + a.tw - 1) / a.tw;
        a.tiles_y = (a.H + a.th - 1) / a.th;
    } else {
        a.lanes = lanes;
        a.tw = lanes - 2 * a.r;
        a.th = rows;   // 0: chosen at launch
        a.tiles_x = (a.W + a.tw - 1) / a.tw;
        a.tiles_y = rows > 0 ? (a.H + rows - 1) / rows : 1;
    }
    return (long long)a.tiles_x * a.tiles_y * a.planes < (1LL << 31) &&
           (long long)a.tiles_x * a.H * a.planes < (1LL << 31);
}

template <int R, int RW>
static hipError_t launch_gs(const GaussLaunch &a, hipStream_t stream) {
    constexpr int CH = gauss_step_rows(R);
    const size_t lds = gauss_stream_lds_bytes(RW, R);
    const void *kern = a.sel ? (const void *)gauss_stream_kernel<R, RW, CH, true>
                             : (const void *)gauss_stream_kernel<R, RW, CH, false>;
    GaussLaunch b = a;
    if (a.th <= 0) {
        // rows per workgroup such that the strips' chunks fill the device's
        // resident workgroup slots once
        static std::atomic<int> slots[2][64];  // per kernel (maps or not) and device; 0 = not yet queried
        const int ks = a.sel ? 1 : 0;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        int n = dev < 64 ? slots[ks][dev].load(std::memory_order_relaxed) : 0;
        if (!n) {
            int cus = 0, per_cu = 0;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, RW, lds);
            if (e != hipSuccess) return e;
            n = std::max(1, cus * per_cu);
            if (dev < 64) slots[ks][dev].store(n, std::memory_order_relaxed);
        }
        const long long strips = (long long)a.tiles_x * a.planes;
        const int per_strip = (int)std::max<long long>(1, n / strips);
        int rows = (a.H + per_strip - 1) / per_strip;
        rows = std::max(CH, (rows + CH - 1) / CH * CH);
        b.th = rows;
        b.tiles_y = (a.H + rows - 1) / rows;
    }
    const int blocks = b.tiles_x * b.tiles_y * b.planes;
    void *args[] = {(void *)&b};
    hipError_t e = hipLaunchKernel(kern, dim3(blocks), dim3(RW), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <int R>
static hipError_t launch_g(const GaussLaunch &a, hipStream_t stream) {
    if (a.lanes == 128) return launch_gs<R, 128>(a, stream);
    if (a.lanes == 256) return launch_gs<R, 256>(a, stream);
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
