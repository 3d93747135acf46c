// Row-streaming forward kernel: one sweep of the exact filter (Alg. 2), of the
// fast approximation (Alg. 3) or of the classical box filter, gfx950.
//
// A workgroup of RW lanes owns a strip of TW output columns (TW a multiple of
// r, TW + 2r <= RW) and a chunk of rows of one plane; lane lx owns region
// column X0 - r + lx.  It walks down the chunk CH rows at a time (a step), so
// the vertical halo is paid once per chunk instead of once per tile, and the
// loads of the next step are in flight while the current one is computed:
//   - the lane's input rows [s - r, s + CH) and its column sums V of the same
//     rows live in registers (the last r rows carry over to the next step);
//     V is formed there in blocks of r rows anchored at multiples of r, with
//     the FP32 operations of the tiled kernels;
//   - the step's V rows and the P rows it evaluates go to LDS, where (row,
//     block of r columns) work items form the row sums Q (into a ring of
//     CH + r rows) and H (of the evaluated rows only);
//   - the lane then evaluates rows [s - r, s + CH - r) of its column, whose
//     windows reach down to row s + CH - 1.
// Each step's stores are issued one step late, ahead of the next step's
// loads (loads and stores share one memory counter, so the wait for those
// loads does not wait on fresh stores).  Two barriers per step.  Every
// running sum restarts at the same image coordinates as in the tiled kernels
// and sums in the same order, so results and maps are bit-identical to them.
#pragma once
#include <algorithm>
#include <atomic>

#include "osbf_device.h"
#include "osbf_fwd_device.h"
#include "osbf_internal.h"

namespace osbf {

// Rows per step for each compiled radius: whole blocks of r rows.  One block
// is fastest (the LDS ring, and with it the workgroups per CU, is smallest),
// except at r <= 2 where the two barriers per step dominate (MI355X,
// 3x2048x2048 FP32).
constexpr int stream_step_rows(int r) {
    return r == 1 ? 2 : r == 2 ? 4 : r;
}

// MODE: MODE_EXACT, MODE_FAST (quadrant means only, no H field) or MODE_BOX,
// as in the tiled kernels; maps (SEL) only with MODE_EXACT.
// One work item t = (plane * chunks + chunk) * strips + strip: rows
// [chunk * th, chunk * th + th) of one strip of one plane (shared by the
// single-image and the batched kernels).
template <int DT, int R, int RW, int CH, bool SEL, int MODE>
__device__ __forceinline__ void fwd_stream_item(FwdLaunch a, int t, float *lds) {
    using S = Storage<DT>;
    using T = typename S::T;
    static_assert(CH % R == 0, "a step is whole blocks of R rows");
    static_assert(RW % 64 == 0 && RW >= 2 * R + R, "region width");
    constexpr int M = CH / R;        // blocks per step
    constexpr int NRB = M + 1;       // blocks in the Q/H ring
    constexpr int PITCH = RW + 1;
    float *const Pl = lds;                      // CH rows: P of the rows evaluated this step
    float *const Vl = lds + CH * PITCH;         // CH rows: V of the step's new rows
    float *const Qr = lds + 2 * CH * PITCH;     // NRB * R rows: ring of Q
    float *const Hr = Qr + NRB * R * PITCH;     // CH rows: H of the rows evaluated this step

    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int ox = X0 - R;
    const int xa = X0, xb = min(W, X0 + TW), xend = xb + R;
    const int yb = min(H, Y0 + YC), yend = yb + R;
    const int lo = max(0, xa - R), hi = min(W, xend) - 1;  // columns the row sums read
    const int x = ox + lx;
    const bool own = x >= xa && x < xb;
    const size_t plane_off = (size_t)plane * H * W;
    // lanes outside the image read a clamped column; their LDS columns are
    // never read (the row sums clamp to [lo, hi])
    const T *src = (const T *)a.src + plane_off + min(max(x, 0), W - 1);
    T *dst = (T *)a.dst + plane_off;
    uint8_t *sel = SEL ? a.sel + plane_off : nullptr;

    // This lane's row-sum work items, the same in every step: items of one
    // block of R rows are consecutive, row fastest, so 32 consecutive lanes
    // read 32 distinct banks (row pitch = 1 mod 32, column blocks R apart)
    // when R divides 32.  CH * nb <= M * RW, so a lane has at most M items.
    const int nb = (xend - xa + R - 1) / R;
    int it_row[M], it_x0[M];
    bool it_ok[M], it_fast[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int it = lx + k * RW;
        const int m = it / (R * nb), rem = it - m * (R * nb);
        const int b = rem / R;
        it_ok[k] = it < CH * nb;
        it_row[k] = m * R + (rem - b * R);
        it_x0[k] = xa + b * R;
        it_fast[k] = it_x0[k] - R >= lo && it_x0[k] + R - 1 <= hi;  // no column clamped
    }

    constexpr float fr1 = (float)(R + 1), f2r1 = (float)(2 * R + 1);
    constexpr float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    float pr[CH + R], vr[CH + R];
    T raw[CH];  // input rows of the next step
#pragma unroll
    for (int i = 0; i < R; ++i) pr[i] = S::cvt(src[(size_t)min(max(Y0 - R + i, 0), H - 1) * W]);
#pragma unroll
    for (int i = 0; i < R; ++i) vr[i] = 0.f;  // rows above Y0: never evaluated
    auto load_step = [&](int s) {
#pragma unroll
        for (int i = 0; i < CH; ++i) raw[i] = src[(size_t)min(max(s + i, 0), H - 1) * W];
    };

    const int nsteps = (yend - Y0 + CH - 1) / CH;
    float out_v[CH];
    int out_i[CH];
    int out_s = 0;
    bool pending = false;
    int base = 0;  // ring block of rows [s - R, s): (n * M) mod NRB
    auto store_step = [&]() {
        auto put = [&](int i) {
            const size_t o = (size_t)(out_s - R + i) * W + x;
            dst[o] = S::pack(out_v[i]);
            if (SEL) sel[o] = (uint8_t)out_i[i];
        };
        if (out_s - R >= Y0 && out_s - R + CH <= yb) {
#pragma unroll
            for (int i = 0; i < CH; ++i) put(i);
        } else {
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (out_s - R + i >= Y0 && out_s - R + i < yb) put(i);
        }
    };
    load_step(Y0);
    for (int n = 0; n < nsteps; ++n) {
        const int s = Y0 + n * CH;
        // V of rows [s, s + CH) from input rows [s - R, s + CH), in registers
#pragma unroll
        for (int i = 0; i < CH; ++i) pr[R + i] = S::cvt(raw[i]);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float *p = pr + m * R;
            float v = p[0];
#pragma unroll
            for (int tt = 1; tt <= R; ++tt) v += p[tt];
            vr[R + m * R] = v;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                v += p[R + tt] - p[tt - 1];
                vr[R + m * R + tt] = v;
            }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            Pl[i * PITCH + lx] = pr[i];  // rows [s - R, s - R + CH), evaluated this step
            Vl[i * PITCH + lx] = vr[R + i];
        }
        // the previous step's results, then the next step's loads
        if (pending && own) store_step();
        if (n + 1 < nsteps) load_step(s + CH);
        __syncthreads();

        // Q of rows [s, s + CH) ∩ [Y0, yend) into ring blocks base + 1 ..
        // base + M, and H of the rows evaluated this step, [s - R, s - R +
        // CH), into Hr; columns [xa, xend).  (An evaluated row y < yb has
        // y + R = s + i < yend, so its item is never skipped.)
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = it_row[k], x0 = it_x0[k];
            if (it_ok[k] && s + i < yend) {
                const float *vrow = Vl + i * PITCH - ox;  // + image column
                const float *prow = Pl + i * PITCH - ox;
                float v[2 * R], p[2 * R];
                if (it_fast[k]) {  // immediate offsets
#pragma unroll
                    for (int tt = 0; tt < 2 * R; ++tt) {
                        v[tt] = vrow[x0 - R + tt];
                        p[tt] = prow[x0 - R + tt];
                    }
                } else {
#pragma unroll
                    for (int tt = 0; tt < 2 * R; ++tt) {
                        const int col = min(max(x0 - R + tt, lo), hi);
                        v[tt] = vrow[col];
                        p[tt] = prow[col];
                    }
                }
                int blk = base + 1 + i / R;
                blk = blk >= NRB ? blk - NRB : blk;
                const int ro = (blk * R + i % R) * PITCH - ox;
                float *qrow = Qr + ro, *hrow = Hr + i * PITCH - ox;
                constexpr bool HF = MODE != MODE_FAST;  // the fast mode needs no H
                float q = v[0], h = p[0];
#pragma unroll
                for (int tt = 1; tt <= R; ++tt) {
                    q += v[tt];
                    if (HF) h += p[tt];
                }
                qrow[x0] = q;
                if (HF) hrow[x0] = h;
                if (x0 + R <= xend) {
#pragma unroll
                    for (int tt = 1; tt < R; ++tt) {
                        q += v[R + tt] - v[tt - 1];
                        qrow[x0 + tt] = q;
                        if (HF) {
                            h += p[R + tt] - p[tt - 1];
                            hrow[x0 + tt] = h;
                        }
                    }
                } else {
#pragma unroll
                    for (int tt = 1; tt < R; ++tt) {
                        if (x0 + tt < xend) {
                            q += v[R + tt] - v[tt - 1];
                            qrow[x0 + tt] = q;
                            if (HF) {
                                h += p[R + tt] - p[tt - 1];
                                hrow[x0 + tt] = h;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();

        // selection and update of rows [s - R, s + CH - R) ∩ [Y0, yb)
        if (own) {
            auto eval_row = [&](int i) {
                int bu = base + i / R;
                bu = bu >= NRB ? bu - NRB : bu;
                const int bd = bu + 1 >= NRB ? bu + 1 - NRB : bu + 1;
                const int ou = (bu * R + i % R) * PITCH + lx;
                const int od = (bd * R + i % R) * PITCH + lx;
                const int oh = i * PITCH + lx;
                const float c = pr[i];
                const float nw = Qr[ou], ne = Qr[ou + R], sw = Qr[od], se = Qr[od + R];
                if constexpr (MODE == MODE_BOX) {
                    out_v[i] = S::round(box_sum(nw, ne, sw, se, Hr[oh], Hr[oh + R], vr[i], vr[i + R], c) * inv_box);
                    out_i[i] = 0;
                } else {
                    float d[8];
                    if constexpr (MODE == MODE_FAST)
                        fast_distances(d, nw, ne, sw, se, c, fr1);
                    else
                        exact_distances(d, nw, ne, sw, se, Hr[oh], Hr[oh + R], vr[i], vr[i + R], c, fr1, f2r1, N);
                    const Pick pk = select8<SEL>(d);
                    out_v[i] = S::round(fmaf(pk.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c));
                    out_i[i] = pk.idx;
                }
            };
            if (s - R >= Y0 && s - R + CH <= yb) {  // uniform over the workgroup
#pragma unroll
                for (int i = 0; i < CH; ++i) eval_row(i);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    if (s - R + i >= Y0 && s - R + i < yb) eval_row(i);
            }
        }
        out_s = s;
        pending = true;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            pr[i] = pr[CH + i];
            vr[i] = vr[CH + i];
        }
        base = base == 0 ? M : base - 1;
    }
    if (pending && own) store_step();
}

// Waves per SIMD the register allocation must leave room for (the LDS ring
// allows about this many workgroups per CU at the default strip widths).
constexpr int stream_min_waves(int r) { return r >= 16 ? 2 : r >= 10 ? 3 : 4; }

template <int DT, int R, int RW, int CH, bool SEL, int MODE = MODE_EXACT>
__global__ __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(stream_min_waves(R))))
void fwd_stream_kernel(FwdLaunch a) {
    extern __shared__ float lds[];
    fwd_stream_item<DT, R, RW, CH, SEL, MODE>(a, xcd_remap(blockIdx.x, a.tiles_x * a.tiles_y * a.planes), lds);
}

template <int DT, int R, int RW, bool SEL, int MODE>
hipError_t launch_stream(const FwdLaunch &a, hipStream_t stream) {
    constexpr int CH = stream_step_rows(R);
    const size_t lds = stream_lds_bytes(RW, R);
    auto kern = fwd_stream_kernel<DT, R, RW, CH, SEL, MODE>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    FwdLaunch b = a;
    if (a.th <= 0) {
        // rows per workgroup chosen so that the strips' chunks fill the
        // device's resident workgroup slots once (no partial last wave)
        static std::atomic<int> slots[64];  // per device; 0 = not yet queried
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        int n = dev < 64 ? slots[dev].load(std::memory_order_relaxed) : 0;
        if (!n) {
            int cus = 0, per_cu = 0;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, RW, lds);
            if (e != hipSuccess) return e;
            n = std::max(1, cus * per_cu);
            if (dev < 64) slots[dev].store(n, std::memory_order_relaxed);
        }
        const long long strips = (long long)a.tiles_x * a.planes;
        const int per_strip = (int)std::max<long long>(1, n / strips);
        int rows = (a.H + per_strip - 1) / per_strip;
        rows = std::max(CH, (rows + CH - 1) / CH * CH);
        b.th = rows;
        b.tiles_y = (a.H + rows - 1) / rows;
    }
    const int blocks = b.tiles_x * b.tiles_y * b.planes;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(RW), lds, stream, b);
    return hipGetLastError();
}

template <int DT, int R, bool SEL, int MODE>
hipError_t launch_stream_w(const FwdLaunch &a, hipStream_t s) {
    switch (a.geom) {
    case GEOM_S128: return launch_stream<DT, R, 128, SEL, MODE>(a, s);
    case GEOM_S192: return launch_stream<DT, R, 192, SEL, MODE>(a, s);
    case GEOM_S256: return launch_stream<DT, R, 256, SEL, MODE>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int DT, bool SEL, int MODE>
hipError_t launch_stream_r(const FwdLaunch &a, hipStream_t s) {
    if (a.k != 1 || !stream_geom(a.geom)) return hipErrorInvalidValue;
    switch (a.r) {
    case 1: return launch_stream_w<DT, 1, SEL, MODE>(a, s);
    case 2: return launch_stream_w<DT, 2, SEL, MODE>(a, s);
    case 3: return launch_stream_w<DT, 3, SEL, MODE>(a, s);
    case 4: return launch_stream_w<DT, 4, SEL, MODE>(a, s);
    case 5: return launch_stream_w<DT, 5, SEL, MODE>(a, s);
    case 8: return launch_stream_w<DT, 8, SEL, MODE>(a, s);
    case 10: return launch_stream_w<DT, 10, SEL, MODE>(a, s);
    case 16: return launch_stream_w<DT, 16, SEL, MODE>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace osbf
