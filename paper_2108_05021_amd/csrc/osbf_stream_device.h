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

// Two fused sweeps on one work item (small radii): stage A runs the first
// sweep on the strip grown by R on each side (rows grown by R), reading the
// input from global memory; its rounded results, still in the lane's
// registers, are stage B's new input rows, from which stage B runs the
// second sweep on the strip itself.  Rows stage B needs above row 0 or below
// row H-1 are replicated from those rows (the clamp), so stage B sees
// exactly the clamp extension of the first sweep's output.  The P and V
// staging and the H rows are shared (stage B's phases follow stage A's after
// barriers), each stage keeps its own Q ring: LDS (5 CH + 2R) rows, four
// barriers per step of CH rows of both sweeps.  The region is TW + 4R
// columns wide.  Every block and column anchor is a multiple of R, so the
// results are those of two single-sweep launches, bit for bit.
template <int DT, int R, int RW, int CH, bool SEL, int MODE>
__device__ __forceinline__ void fwd_stream2_item(const FwdLaunch &a, int t, float *lds) {
    using S = Storage<DT>;
    using T = typename S::T;
    static_assert(CH % R == 0, "a step is whole blocks of R rows");
    static_assert(RW % 64 == 0 && RW >= 5 * R, "region width");
    constexpr int M = CH / R, NRB = M + 1, PITCH = RW + 1;
    float *const Pl = lds;                          // CH rows
    float *const Vl = lds + CH * PITCH;             // CH rows
    float *const Hr = lds + 2 * CH * PITCH;         // CH rows
    float *const QA = lds + 3 * CH * PITCH;         // NRB * R rows (stage A ring)
    float *const QB = QA + NRB * R * PITCH;         // NRB * R rows (stage B ring)

    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int yb = min(H, Y0 + YC);
    const int ox = X0 - 2 * R;  // image column of region column 0
    const int x = ox + lx;
    const size_t plane_off = (size_t)plane * H * W;
    const T *src = (const T *)a.src + plane_off + min(max(x, 0), W - 1);
    T *dst = (T *)a.dst + plane_off;
    uint8_t *selA = SEL ? a.sel + plane_off : nullptr;
    uint8_t *selB = SEL ? a.sel + a.sel_stride + plane_off : nullptr;

    // stage geometry: evaluated columns [xa, xb) and rows [ya, ye), fields
    // on columns [xa, xend) and rows up to yend, row sums reading [lo, hi]
    struct Geo { int xa, xb, xend, lo, hi, ya, ye, yend, nb; };
    auto geo = [&](int xa, int xb, int ya, int ye) {
        Geo g;
        g.xa = xa; g.xb = xb; g.xend = xb + R;
        g.lo = max(0, xa - R); g.hi = min(W, g.xend) - 1;
        g.ya = ya; g.ye = ye; g.yend = ye + R;
        g.nb = (g.xend - xa + R - 1) / R;
        return g;
    };
    const Geo gA = geo(max(0, X0 - R), min(W, X0 + TW + R), max(0, Y0 - R), min(H, yb + R));
    const Geo gB = geo(X0, min(W, X0 + TW), Y0, yb);
    const bool ownA = x >= gA.xa && x < gA.xb, ownB = x >= gB.xa && x < gB.xb;
    const bool coreA = x >= X0 && x < X0 + TW;  // stage A writes maps only here

    // each stage's row-sum items, the same every step (as fwd_stream_item)
    struct Items { int row[M], x0[M]; bool ok[M], fast[M]; };
    auto items = [&](const Geo &g) {
        Items it;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = lx + k * RW;
            const int m = i / (R * g.nb), rem = i - m * (R * g.nb);
            const int b = rem / R;
            it.ok[k] = i < CH * g.nb;
            it.row[k] = m * R + (rem - b * R);
            it.x0[k] = g.xa + b * R;
            it.fast[k] = it.x0[k] - R >= g.lo && it.x0[k] + R - 1 <= g.hi;
        }
        return it;
    };
    const Items iA = items(gA), iB = items(gB);

    constexpr float fr1 = (float)(R + 1), f2r1 = (float)(2 * R + 1);
    constexpr float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    float prA[CH + R], vrA[CH + R], prB[CH + R], vrB[CH + R];
    float outA[CH], outB[CH];
    int idxA[CH], idxB[CH];
    T raw[CH];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        prA[i] = S::cvt(src[(size_t)min(max(gA.ya - R + i, 0), H - 1) * W]);
        vrA[i] = prB[i] = vrB[i] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) outA[i] = outB[i] = 0.f;
    auto load_step = [&](int s0) {
#pragma unroll
        for (int i = 0; i < CH; ++i) raw[i] = src[(size_t)min(max(s0 + i, 0), H - 1) * W];
    };

    // V of the step's new rows in registers; P of the rows evaluated this step
    // and the new V rows to LDS
    auto v_phase = [&](float *pr, float *vr) {
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
            Pl[i * PITCH + lx] = pr[i];
            Vl[i * PITCH + lx] = vr[R + i];
        }
    };
    // Q of rows [s, s + CH) into the ring, H of rows [s - R, s - R + CH)
    auto qh_phase = [&](const Geo &g, const Items &it, int s0, int base, float *Q) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = it.row[k], x0 = it.x0[k];
            if (!it.ok[k] || s0 + i >= g.yend) continue;
            const float *vrow = Vl + i * PITCH - ox;  // + image column
            const float *prow = Pl + i * PITCH - ox;
            float v[2 * R], p[2 * R];
            if (it.fast[k]) {
#pragma unroll
                for (int tt = 0; tt < 2 * R; ++tt) {
                    v[tt] = vrow[x0 - R + tt];
                    p[tt] = prow[x0 - R + tt];
                }
            } else {
#pragma unroll
                for (int tt = 0; tt < 2 * R; ++tt) {
                    const int col = min(max(x0 - R + tt, g.lo), g.hi);
                    v[tt] = vrow[col];
                    p[tt] = prow[col];
                }
            }
            int blk = base + 1 + i / R;
            blk = blk >= NRB ? blk - NRB : blk;
            float *qrow = Q + (blk * R + i % R) * PITCH - ox, *hrow = Hr + i * PITCH - ox;
            constexpr bool HF = MODE != MODE_FAST;
            float q = v[0], h = p[0];
#pragma unroll
            for (int tt = 1; tt <= R; ++tt) {
                q += v[tt];
                if (HF) h += p[tt];
            }
            qrow[x0] = q;
            if (HF) hrow[x0] = h;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (x0 + tt < g.xend) {
                    q += v[R + tt] - v[tt - 1];
                    qrow[x0 + tt] = q;
                    if (HF) {
                        h += p[R + tt] - p[tt - 1];
                        hrow[x0 + tt] = h;
                    }
                }
            }
        }
    };
    // rows [s - R, s - R + CH) ∩ [ya, ye) of this lane's column
    auto eval_phase = [&](const Geo &g, int s0, int base, const float *Q, const float *pr, const float *vr,
                          float *out, int *idx) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int y = s0 - R + i;
            if (y < g.ya || y >= g.ye) continue;  // uniform over the workgroup
            int bu = base + i / R;
            bu = bu >= NRB ? bu - NRB : bu;
            const int bd = bu + 1 >= NRB ? bu + 1 - NRB : bu + 1;
            const int ou = (bu * R + i % R) * PITCH + lx;
            const int od = (bd * R + i % R) * PITCH + lx;
            const int oh = i * PITCH + lx;
            const float c = pr[i];
            const float nw = Q[ou], ne = Q[ou + R], sw = Q[od], se = Q[od + R];
            if constexpr (MODE == MODE_BOX) {
                out[i] = S::round(box_sum(nw, ne, sw, se, Hr[oh], Hr[oh + R], vr[i], vr[i + R], c) * inv_box);
                idx[i] = 0;
            } else {
                float d[8];
                if constexpr (MODE == MODE_FAST)
                    fast_distances(d, nw, ne, sw, se, c, fr1);
                else
                    exact_distances(d, nw, ne, sw, se, Hr[oh], Hr[oh + R], vr[i], vr[i + R], c, fr1, f2r1, N);
                const Pick pk = select8<SEL>(d);
                out[i] = S::round(fmaf(pk.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c));
                idx[i] = pk.idx;
            }
        }
    };

    const int nsteps = (yb + 2 * R - gA.ya + CH - 1) / CH;
    int baseA = 0, baseB = 0, outB_s = 0;
    bool pending = false;
    auto store_B = [&]() {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int y = outB_s - R + i;
            if (y >= Y0 && y < yb) {
                const size_t o = (size_t)y * W + x;
                dst[o] = S::pack(outB[i]);
                if (SEL) selB[o] = (uint8_t)idxB[i];
            }
        }
    };
    load_step(gA.ya);
    for (int n = 0; n < nsteps; ++n) {
        const int sA = gA.ya + n * CH, sB = sA - R;
        // stage A: the first sweep from the input
#pragma unroll
        for (int i = 0; i < CH; ++i) prA[R + i] = S::cvt(raw[i]);
        v_phase(prA, vrA);
        if (pending && ownB) store_B();
        if (n + 1 < nsteps) load_step(sA + CH);
        __syncthreads();
        qh_phase(gA, iA, sA, baseA, QA);
        __syncthreads();
        if (ownA) {
            eval_phase(gA, sA, baseA, QA, prA, vrA, outA, idxA);
            if (SEL && coreA) {
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int y = sA - R + i;
                    if (y >= Y0 && y < yb) selA[(size_t)y * W + x] = (uint8_t)idxA[i];
                }
            }
        }
        // stage B: its new rows [sB, sB + CH) are stage A's rows just
        // evaluated; rows outside the image repeat row 0 or row H - 1
#pragma unroll
        for (int i = 0; i < CH; ++i) prB[R + i] = outA[i];
        {
            const int j0 = R - sB, jH = H - 1 + R - sB;  // window indices of rows 0 and H - 1
            if (j0 > 0 && j0 < R + CH) {  // uniform
                const float v0 = prB[0];
                float top = v0;
#pragma unroll
                for (int j = 0; j < R + CH; ++j)
                    if (j == j0) top = prB[j];
#pragma unroll
                for (int j = 0; j < R + CH; ++j)
                    if (j < j0) prB[j] = top;
            }
            if (jH >= 0 && jH < R + CH - 1) {  // uniform
                float bot = prB[0];
#pragma unroll
                for (int j = 0; j < R + CH; ++j)
                    if (j == jH) bot = prB[j];
#pragma unroll
                for (int j = 0; j < R + CH; ++j)
                    if (j > jH) prB[j] = bot;
            }
        }
        v_phase(prB, vrB);
        __syncthreads();
        qh_phase(gB, iB, sB, baseB, QB);
        __syncthreads();
        if (ownB) eval_phase(gB, sB, baseB, QB, prB, vrB, outB, idxB);
        outB_s = sB;
        pending = true;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            prA[i] = prA[CH + i];
            vrA[i] = vrA[CH + i];
            prB[i] = prB[CH + i];
            vrB[i] = vrB[CH + i];
        }
        baseA = baseA == 0 ? M : baseA - 1;
        baseB = baseB == 0 ? M : baseB - 1;
    }
    if (pending && ownB) store_B();
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

// Radii with a fused two-sweep streaming kernel (halo 2r per side).
constexpr bool stream2_radius(int r) { return r <= 5; }

template <int DT, int R, int RW, int CH, bool SEL, int MODE = MODE_EXACT>
__global__ __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(stream_min_waves(R))))
void fwd_stream2_kernel(FwdLaunch a) {
    extern __shared__ float lds[];
    fwd_stream2_item<DT, R, RW, CH, SEL, MODE>(a, xcd_remap(blockIdx.x, a.tiles_x * a.tiles_y * a.planes), lds);
}

template <int DT, int R, int RW, bool SEL, int MODE>
hipError_t launch_stream(const FwdLaunch &a, hipStream_t stream) {
    constexpr int CH = stream_step_rows(R);
    const bool fused = a.k == 2;
    if constexpr (!stream2_radius(R) || RW < 5 * R) {
        if (fused) return hipErrorInvalidValue;
    }
    const size_t lds = fused ? stream2_lds_bytes(RW, R) : stream_lds_bytes(RW, R);
    const void *kern = (const void *)fwd_stream_kernel<DT, R, RW, CH, SEL, MODE>;
    if constexpr (stream2_radius(R) && RW >= 5 * R) {
        if (fused) kern = (const void *)fwd_stream2_kernel<DT, R, RW, CH, SEL, MODE>;
    }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    FwdLaunch b = a;
    if (a.th <= 0) {
        // rows per workgroup chosen so that the strips' chunks fill the
        // device's resident workgroup slots once (no partial last wave)
        static std::atomic<int> slots[2][64];  // per kernel and device; 0 = not yet queried
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        int n = dev < 64 ? slots[fused][dev].load(std::memory_order_relaxed) : 0;
        if (!n) {
            int cus = 0, per_cu = 0;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, RW, lds);
            if (e != hipSuccess) return e;
            n = std::max(1, cus * per_cu);
            if (dev < 64) slots[fused][dev].store(n, std::memory_order_relaxed);
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
    if (a.k < 1 || a.k > 2 || !stream_geom(a.geom)) return hipErrorInvalidValue;
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
