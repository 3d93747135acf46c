// Classical box filter, the baseline the paper times its filter against
// (Sec. III-G, Table I): one sweep replaces every pixel by the mean of the
// full (2r+1) x (2r+1) window of the replicate extension, gfx950.
//
// Separable, two passes on one work item (a strip of TW output columns and a
// chunk of rows of one plane, walked CH rows per step):
//   vertical    B(x, y) = sum_{y'=y-r..y+r} P(x, y'), per lane (lane = column)
//               in registers: a direct sum of 2r+1 rows where y is a multiple
//               of r, then r-1 slides;
//   horizontal  S(x, y) = sum_{x'=x-r..x+r} B(x', y), from the B rows staged
//               in LDS, by (row, block of r columns) work items: a direct sum
//               at the block start, then slides;
// then each lane scales its column of S by 1/(2r+1)^2 and stores it one step
// later, ahead of the next step's loads (loads and stores share one memory
// counter).  Lanes outside the image hold the clamped column, so the
// horizontal sums need no index clamping.  LDS: the B and S rows of a step.
// No window selection, no quadrant field: a minimal separable filter.
#include <algorithm>
#include <atomic>

#include "osbf_device.h"
#include "osbf_internal.h"

namespace osbf {

constexpr int box_step_rows(int r) { return r == 1 ? 4 : r == 2 ? 4 : r; }
constexpr int box_gcd(int a, int b) { return b == 0 ? a : box_gcd(b, a % b); }
constexpr int kBoxLanes = 128;

template <int DT, int R>
__global__ __launch_bounds__(kBoxLanes) void box_stream_kernel(BoxLaunch a) {
    using S = Storage<DT>;
    using T = typename S::T;
    constexpr int RW = kBoxLanes, CH = box_step_rows(R), PITCH = RW + 1;
    constexpr int LP = 2 * R + CH;  // P rows [s - 2R, s + CH) of the step
    static_assert(CH % R == 0, "a step is whole blocks of R rows");
    extern __shared__ float lds[];
    float *const Bs = lds;                // CH rows: vertical sums of the step's output rows
    float *const Ss = lds + CH * PITCH;   // CH rows: their horizontal sums

    const int t = xcd_remap(blockIdx.x, a.tiles_x * a.tiles_y * a.planes);
    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int ox = X0 - R;  // image column of lane 0
    const int xb = min(W, X0 + TW), yb = min(H, Y0 + YC);
    const int x = ox + lx;
    const bool own = x >= X0 && x < xb;
    // output rows [s - R, s - R + CH) per step; the first step fills the ring
    const int nsteps = (yb + R - Y0 + CH - 1) / CH;
    const int es = (int)sizeof(T), rowb = W * es;
    const int row0 = max(0, Y0 - 2 * R);
    const int row1 = min(H, Y0 + nsteps * CH);
    BufRsrc src, dst;
    {
        const size_t first = (size_t)plane * H * W + (size_t)row0 * W;
        const uint32_t n = (uint32_t)(row1 - row0) * (uint32_t)W * es;
        src = buf_rsrc((const T *)a.src + first, n);
        dst = buf_rsrc((T *)a.dst + first, n);
    }
    const int vld = clampi(x, 0, W - 1) * es, vst = x * es;
    auto ld = [&](int y) { return S::load_raw(src, vld, (clampi(y, 0, H - 1) - row0) * rowb); };

    // this lane's horizontal work items (as in the forward's row sums)
    constexpr int M = CH / R;
    const int nb = (xb - X0 + R - 1) / R;
    int it_row[M], it_ib[M];
    bool it_ok[M], it_full[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int it = lx + k * RW;
        const int m = it / (R * nb), rem = it - m * (R * nb);
        const int b = rem / R;
        it_ok[k] = it < CH * nb;
        it_row[k] = m * R + (rem - b * R);
        const int x0 = X0 + b * R;
        it_ib[k] = x0 - R - ox;  // LDS column of the item's first read
        it_full[k] = x0 + R <= xb;
    }
    constexpr float inv = 1.0f / (float)((2 * R + 1) * (2 * R + 1));

    float PR[LP];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) PR[j] = S::from_raw(ld(Y0 - 2 * R + j));
#pragma unroll
    for (int j = 0; j < CH; ++j) PR[2 * R + j] = ld(Y0 + j);
    float out[CH];
    int out_s = 0;
    bool pending = false;

    auto store_prev = [&]() {
        if (out_s - R >= Y0 && out_s - R + CH <= yb) {  // uniform
            int o = (out_s - R - row0) * rowb;
#pragma unroll
            for (int i = 0; i < CH; ++i, o += rowb) S::store_bits(dst, vst, o, out[i]);
        } else {
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int y = out_s - R + i;
                if (y >= Y0 && y < yb) S::store_bits(dst, vst, (y - row0) * rowb, out[i]);
            }
        }
    };

    auto step = [&](auto ph, int n) {
        constexpr int PH = decltype(ph)::value;
        auto sl = [](int j) { return (j + PH * CH) % LP; };  // logical j <-> row s - 2R + j
        const int s = Y0 + n * CH;
#pragma unroll
        for (int j = 2 * R; j < LP; ++j) PR[sl(j)] = S::from_raw(PR[sl(j)]);
        // vertical sums of output rows [s - R, s - R + CH): blocks of R rows
#pragma unroll
        for (int m = 0; m < M; ++m) {
            float v = PR[sl(m * R)];
#pragma unroll
            for (int tt = 1; tt <= 2 * R; ++tt) v += PR[sl(m * R + tt)];
            Bs[(m * R) * PITCH + lx] = v;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                v += PR[sl(m * R + tt + 2 * R)] - PR[sl(m * R + tt - 1)];
                Bs[(m * R + tt) * PITCH + lx] = v;
            }
        }
        if (pending && own) store_prev();
        if (n + 1 < nsteps) {  // the next step's rows into the slots of rows [s - 2R, s - 2R + CH)
            if (s + 2 * CH <= H) {
                int o = (s + CH - row0) * rowb;
#pragma unroll
                for (int i = 0; i < CH; ++i, o += rowb) PR[sl(i)] = S::load_raw(src, vld, o);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i) PR[sl(i)] = ld(s + CH + i);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = it_row[k];
            if (!it_ok[k]) continue;
            const float *b = Bs + i * PITCH + it_ib[k];  // columns x0 - R ..
            float *o = Ss + i * PITCH + it_ib[k] + R;
            float v[3 * R];
#pragma unroll
            for (int tt = 0; tt < 3 * R; ++tt) v[tt] = b[tt];
            float q = v[0];
#pragma unroll
            for (int tt = 1; tt <= 2 * R; ++tt) q += v[tt];
            o[0] = q;
            const int x0 = it_ib[k] + R + ox;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (it_full[k] || x0 + tt < xb) {
                    q += v[tt + 2 * R] - v[tt - 1];
                    o[tt] = q;
                }
            }
        }
        __syncthreads();
        if (own) {
#pragma unroll
            for (int i = 0; i < CH; ++i) out[i] = S::bits(Ss[i * PITCH + lx] * inv);
        }
        out_s = s;
        pending = true;
    };

    constexpr int NPH = LP / box_gcd(LP, CH);  // ring period in steps
    static_assert((NPH * CH) % LP == 0, "ring period");
    for (int n = 0; n < nsteps; n += NPH) {
        static_for<0, NPH>([&](auto ph) {
            if (n + decltype(ph)::value < nsteps) step(ph, n + decltype(ph)::value);
        });
    }
    if (pending && own) store_prev();
}

size_t box_lds_bytes(int r) { return (size_t)2 * box_step_rows(r) * (kBoxLanes + 1) * sizeof(float); }

bool box_radius(int r) { return r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 10 || r == 16; }

void box_geometry(int r, int *tw, int *step) {
    *tw = ((kBoxLanes - 2 * r) / r) * r;
    *step = box_step_rows(r);
}

template <int DT, int R>
static hipError_t launch_box_r(const BoxLaunch &a, hipStream_t stream) {
    const void *kern = (const void *)box_stream_kernel<DT, R>;
    const size_t lds = box_lds_bytes(R);
    BoxLaunch b = a;
    // rows per workgroup: the strips' chunks fill the resident workgroup
    // slots once (as the forward's streaming kernel)
    static std::atomic<int> slots[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int n = dev < 64 ? slots[dev].load(std::memory_order_relaxed) : 0;
    if (!n) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBoxLanes, lds);
        if (e != hipSuccess) return e;
        n = std::max(1, cus * per_cu);
        if (dev < 64) slots[dev].store(n, std::memory_order_relaxed);
    }
    constexpr int CH = box_step_rows(R);
    const long long strips = (long long)a.tiles_x * a.planes;
    const int per_strip = (int)std::max<long long>(1, n / strips);
    int rows = (a.H + per_strip - 1) / per_strip;
    rows = std::max(CH, (rows + CH - 1) / CH * CH);
    const long long row_bytes = (long long)a.W * (DT == DT_F32 ? 4 : 2);
    auto fits = [&](long long rr) { return (rr + 4 * R + 2 * CH) * row_bytes < (1LL << 31); };
    while (rows > CH && !fits(rows)) rows = std::max(CH, rows / 2 / CH * CH);
    if (!fits(rows)) return hipErrorInvalidValue;
    b.th = rows;
    b.tiles_y = (a.H + rows - 1) / rows;
    const long long blocks = (long long)b.tiles_x * b.tiles_y * b.planes;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    void *args[] = {(void *)&b};
    e = hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(kBoxLanes), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_box_dt(const BoxLaunch &a, hipStream_t s) {
    switch (a.r) {
    case 1: return launch_box_r<DT, 1>(a, s);
    case 2: return launch_box_r<DT, 2>(a, s);
    case 3: return launch_box_r<DT, 3>(a, s);
    case 4: return launch_box_r<DT, 4>(a, s);
    case 5: return launch_box_r<DT, 5>(a, s);
    case 8: return launch_box_r<DT, 8>(a, s);
    case 10: return launch_box_r<DT, 10>(a, s);
    case 16: return launch_box_r<DT, 16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_box(int dtype, const BoxLaunch &a, hipStream_t s) {
    switch (dtype) {
    case DT_F32: return launch_box_dt<DT_F32>(a, s);
    case DT_F16: return launch_box_dt<DT_F16>(a, s);
    default: return launch_box_dt<DT_BF16>(a, s);
    }
}

}  // namespace osbf
