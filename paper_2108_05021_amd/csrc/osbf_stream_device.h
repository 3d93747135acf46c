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

// Rows per step for each compiled radius: whole blocks of r rows, or a
// whole fraction of one.  One block is fastest from r = 3 to 10 (the LDS
// ring, and with it the workgroups per CU, is smallest), two at r <= 2 where
// the two barriers per step dominate (MI355X, 3x2048x2048 FP32); half a
// block at r = 16, whose LDS then fits three workgroups per CU instead of
// two (1x8192x8192: 5% faster).
constexpr int stream_step_rows(int r) {
    return r == 1 ? 2 : r == 2 ? 4 : r == 16 ? 8 : r;
}

// Register (and Q) ring rows for r and CH rows per step.  Steps of whole
// blocks keep the rows [s - r, s + CH); steps of part of a block also keep
// row s - r - 1 (a block's later steps continue its running column sums,
// which drop that row), rounded up to whole blocks so that the ring's period
// in steps is a whole number of blocks.
constexpr int stream_ring_rows(int r, int ch) {
    return ch >= r ? r + ch : (r + 1 + ch + r - 1) / r * r;
}

constexpr int stream_gcd(int a, int b) { return b == 0 ? a : stream_gcd(b, a % b); }

// Rows per work item are a multiple of this (whole steps and whole blocks).
constexpr int stream_row_quantum(int r) {
    return stream_step_rows(r) > r ? stream_step_rows(r) : r;
}

// Rows [row0, row1) of one plane that a work item touches, as buffer
// resources of the iterate (and of the map): every access is a 32-bit lane
// offset plus a scalar row offset from row0.  The iterate's rows may be
// strided (src and dst each their own row and plane strides); maps are
// contiguous.
struct ItemRows {
    BufRsrc src, dst, sel;
    int row0, H, W;
    int srow, drow;  // bytes per row of the iterate read / written
    __device__ __forceinline__ int ld_off(int y) const { return (clampi(y, 0, H - 1) - row0) * srow; }
    __device__ __forceinline__ int st_off(int y) const { return (y - row0) * drow; }
    __device__ __forceinline__ int sel_off(int y) const { return (y - row0) * W; }
};

template <typename T>
__device__ __forceinline__ ItemRows item_rows(const FwdLaunch &a, int plane, int row0, int row1, bool sel) {
    ItemRows io;
    io.H = a.H;
    io.W = a.W;
    io.row0 = row0;
    const int sld = a.src_ld ? a.src_ld : a.W, dld = a.dst_ld ? a.dst_ld : a.W;
    const long long sps = a.src_ps ? a.src_ps : (long long)a.H * a.W;
    const long long dps = a.dst_ps ? a.dst_ps : (long long)a.H * a.W;
    io.srow = sld * (int)sizeof(T);
    io.drow = dld * (int)sizeof(T);
    const uint32_t nr = (uint32_t)(row1 - row0);
    io.src = buf_rsrc((const T *)a.src + plane * sps + (long long)row0 * sld, nr * (uint32_t)io.srow);
    io.dst = buf_rsrc((T *)a.dst + plane * dps + (long long)row0 * dld, nr * (uint32_t)io.drow);
    io.sel = sel ? buf_rsrc(a.sel + (size_t)plane * a.H * a.W + (size_t)row0 * a.W, nr * (uint32_t)a.W) : io.dst;
    return io;
}

// MODE: MODE_EXACT, MODE_FAST (quadrant means only, no H field) or MODE_BOX,
// as in the tiled kernels; maps (SEL) only with MODE_EXACT.
// One work item t = (plane * chunks + chunk) * strips + strip: rows
// [chunk * th, chunk * th + th) of one strip of one plane (shared by the
// single-image and the batched kernels).
//
// Registers: the lane's P and V rows [s - R, s + CH) (from s - R - 1 when a
// step is part of a block) sit in two rings of L registers whose origin
// advances by CH rows per step, so the step body is unrolled over the ring
// period NRB and every ring slot, every slot of the Q ring in LDS and every
// LDS offset is a compile-time constant.  The next step's rows are loaded
// straight into ring slots of rows no longer needed once the step's rows are
// staged in LDS (the evaluation reads c from LDS).  Lanes outside the image hold the clamped column, so the
// row sums read the replicate extension without clamping indices.
template <int DT, int R, int RW, int CH, bool SEL, int MODE>
__device__ __forceinline__ void fwd_stream_item(const FwdLaunch &a, int t, float *lds) {
    using S = Storage<DT>;
    using T = typename S::T;
    static_assert(CH % R == 0 || R % CH == 0, "a step is whole blocks of R rows or a whole part of one");
    static_assert(RW % 64 == 0 && RW >= 2 * R + R, "region width");
    constexpr int M = CH >= R ? CH / R : 1;     // blocks per step (at least one row-sum item per lane)
    constexpr int MB = CH >= R ? 1 : R / CH;    // steps per block
    constexpr int RB = CH >= R ? R : CH;        // rows of one block within a step
    constexpr int OFF = MB == 1 ? R : R + 1;    // ring rows above the step's first new row
    constexpr int L = stream_ring_rows(R, CH);  // register ring length, also the Q ring's
    constexpr int NRB = L / stream_gcd(L, CH);  // ring period in steps (a multiple of MB)
    static_assert(L >= OFF + CH && NRB % MB == 0, "ring");
    constexpr int PITCH = RW + 1;
    // staging, CH blocks of three rows: P of the i-th row evaluated this step
    // (row s - R + i), V of the step's i-th new row (row s + i), H of the
    // i-th evaluated row; then the ring of Q (L rows, R + CH of them in use).  Block stride = 1 mod
    // 32 banks, as the ring's pitch, so that the row-sum items (consecutive
    // lanes = consecutive rows of one block of columns) hit distinct banks.
    constexpr int RS = 3 * PITCH + 30;
    float *const Sg = lds;
    float *const Qr = lds + CH * RS;

    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int ox = X0 - R;
    const int xa = X0, xb = min(W, X0 + TW), xend = xb + R;
    const int yb = min(H, Y0 + YC), yend = yb + R;
    const int x = ox + lx;
    const bool own = x >= xa && x < xb;
    const int nsteps = (yend - Y0 + CH - 1) / CH;

    // rows up to the last one loaded or stored
    const ItemRows io = item_rows<T>(a, plane, max(0, Y0 - OFF), min(H, Y0 + nsteps * CH), SEL);
    const int vld = clampi(x, 0, W - 1) * (int)sizeof(T);  // this lane's column (clamped)
    const int vst = x * (int)sizeof(T);

    // This lane's row-sum work items, the same in every step: items of the
    // step's rows of one block of R rows are consecutive, row fastest, so 32
    // consecutive lanes read 32 distinct banks (row pitch = 1 mod 32, column
    // blocks R apart) when R divides 32.  CH * nb <= M * RW, so a lane has at
    // most M items.
    // ib: the item's first LDS column in its row, relative to the row start.
    const int nb = (xend - xa + R - 1) / R;
    int it_row[M], it_ib[M];
    bool it_ok[M], it_full[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int it = lx + k * RW;
        const int m = it / (RB * nb), rem = it - m * (RB * nb);
        const int b = rem / RB;
        it_ok[k] = it < CH * nb;
        it_row[k] = m * RB + (rem - b * RB);
        const int x0 = xa + b * R;
        it_ib[k] = x0 - R - ox;
        it_full[k] = x0 + R <= xend;
    }

    constexpr float fr1 = (float)(R + 1), f2r1 = (float)(2 * R + 1);
    constexpr float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    float PR[L], VR[L];  // physical rings
#pragma unroll
    for (int j = 0; j < OFF; ++j) {
        PR[j] = S::from_raw(S::load_raw(io.src, vld, io.ld_off(Y0 - OFF + j)));
        VR[j] = 0.f;  // rows above Y0: never evaluated
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) PR[OFF + j] = S::load_raw(io.src, vld, io.ld_off(Y0 + j));

    float out_v[CH];
    int out_i[CH];
    int out_s = 0;
    bool pending = false;
    auto store_step = [&]() {
        auto put = [&](int i) {
            const int y = out_s - R + i;
            S::store_bits(io.dst, vst, io.st_off(y), out_v[i]);
            if (SEL) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)out_i[i], io.sel, x, io.sel_off(y), 0);
        };
        if (out_s - R >= Y0 && out_s - R + CH <= yb) {  // uniform: offsets step by a row
            int o = io.st_off(out_s - R), os = io.sel_off(out_s - R);
#pragma unroll
            for (int i = 0; i < CH; ++i, o += io.drow, os += W) {
                S::store_bits(io.dst, vst, o, out_v[i]);
                if (SEL) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)out_i[i], io.sel, x, os, 0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (out_s - R + i >= Y0 && out_s - R + i < yb) put(i);
        }
    };

    auto step = [&](auto ph, int n) {
        constexpr int PH = decltype(ph)::value;
        // physical slot of logical ring row j (row s - OFF + j)
        auto sl = [](int j) { return (j + PH * CH) % L; };
        // Q ring row of image row s + j, j in [-R, CH)
        auto qrow = [](int j) { return (PH * CH + R + j) % L; };
        const int s = Y0 + n * CH;
        wave_priority<1>();
        // V of rows [s, s + CH) from P rows [s - R - 1, s + CH), in registers:
        // at a block's first row a direct sum of R + 1 rows, then slides
#pragma unroll
        for (int j = OFF; j < OFF + CH; ++j) PR[sl(j)] = S::from_raw(PR[sl(j)]);
        if constexpr (MB == 1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float v = PR[sl(m * R)];
#pragma unroll
                for (int tt = 1; tt <= R; ++tt) v += PR[sl(m * R + tt)];
                VR[sl(R + m * R)] = v;
#pragma unroll
                for (int tt = 1; tt < R; ++tt) {
                    v += PR[sl(R + m * R + tt)] - PR[sl(m * R + tt - 1)];
                    VR[sl(R + m * R + tt)] = v;
                }
            }
        } else {
            float v;
            int t0 = 0;
            if constexpr (PH % MB == 0) {  // the step starts a block
                v = PR[sl(OFF - R)];
#pragma unroll
                for (int tt = 1; tt <= R; ++tt) v += PR[sl(OFF - R + tt)];
                VR[sl(OFF)] = v;
                t0 = 1;
            } else {
                v = VR[sl(OFF - 1)];  // the block's running sum at row s - 1
            }
#pragma unroll
            for (int tt = t0; tt < CH; ++tt) {
                v += PR[sl(OFF + tt)] - PR[sl(OFF + tt - R - 1)];
                VR[sl(OFF + tt)] = v;
            }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            Sg[i * RS + lx] = PR[sl(OFF - R + i)];  // rows [s - R, s - R + CH), evaluated this step
            Sg[i * RS + PITCH + lx] = VR[sl(OFF + i)];
        }
        // the previous step's results, then the next step's loads into the
        // slots of rows no longer needed (for whole-block steps, the rows just
        // staged)
        if (pending && own) store_step();
        if (n + 1 < nsteps) {
            if (s + 2 * CH <= H) {  // uniform: no clamped row, offsets step by a row
                int o = io.ld_off(s + CH);
#pragma unroll
                for (int i = 0; i < CH; ++i, o += io.srow) PR[sl(OFF + CH + i)] = S::load_raw(io.src, vld, o);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i) PR[sl(OFF + CH + i)] = S::load_raw(io.src, vld, io.ld_off(s + CH + i));
            }
        }
        __syncthreads();
        wave_priority<2>();

        // Q of rows [s, s + CH) ∩ [Y0, yend) into the ring and H of the rows
        // evaluated this step, [s - R, s - R + CH), into Hr; columns [xa, xend).
        // (An evaluated row y < yb has y + R = s + i < yend, so its item is
        // never skipped.)
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = it_row[k];
            if (it_ok[k] && s + i < yend) {
                const int ib = i * RS + it_ib[k];
                float v[2 * R], p[2 * R];
#pragma unroll
                for (int tt = 0; tt < 2 * R; ++tt) {
                    p[tt] = Sg[ib + tt];
                    v[tt] = Sg[ib + PITCH + tt];
                }
                int qo;
                if constexpr (M == 1) {
                    qo = qrow(0) * PITCH + it_ib[k] + R;  // qrow(0) a multiple of CH, i < CH: no wrap
                    qo += i * PITCH;
                } else {
                    const int qr = (PH * CH + R) % L + i;
                    qo = (qr >= L ? qr - L : qr) * PITCH + it_ib[k] + R;
                }
                float *qrow_p = Qr + qo;
                float *hrow_p = Sg + ib + 2 * PITCH + R;
                constexpr bool HF = MODE != MODE_FAST;  // the fast mode needs no H
                float q = v[0], h = p[0];
#pragma unroll
                for (int tt = 1; tt <= R; ++tt) {
                    q += v[tt];
                    if (HF) h += p[tt];
                }
                qrow_p[0] = q;
                if (HF) hrow_p[0] = h;
                if (it_full[k]) {
#pragma unroll
                    for (int tt = 1; tt < R; ++tt) {
                        q += v[R + tt] - v[tt - 1];
                        qrow_p[tt] = q;
                        if (HF) {
                            h += p[R + tt] - p[tt - 1];
                            hrow_p[tt] = h;
                        }
                    }
                } else {
                    const int x0 = it_ib[k] + R + ox;
#pragma unroll
                    for (int tt = 1; tt < R; ++tt) {
                        if (x0 + tt < xend) {
                            q += v[R + tt] - v[tt - 1];
                            qrow_p[tt] = q;
                            if (HF) {
                                h += p[R + tt] - p[tt - 1];
                                hrow_p[tt] = h;
                            }
                        }
                    }
                }
            }
        }
        wave_priority<0>();
        __syncthreads();

        // selection and update of rows [s - R, s + CH - R) ∩ [Y0, yb)
        if (own) {
            auto eval_row = [&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int ou = qrow(i - R) * PITCH, od = qrow(i) * PITCH, op = i * RS, oh = op + 2 * PITCH;
                const float c = Sg[op + lx];
                const float nw = Qr[ou + lx], ne = Qr[ou + lx + R], sw = Qr[od + lx], se = Qr[od + lx + R];
                const float vu = VR[sl(OFF - R + i)], vd = VR[sl(OFF + i)];
                if constexpr (MODE == MODE_BOX) {
                    out_v[i] = S::bits(box_sum(nw, ne, sw, se, Sg[oh + lx], Sg[oh + lx + R], vu, vd, c) * inv_box);
                    out_i[i] = 0;
                } else {
                    float d[8];
                    if constexpr (MODE == MODE_FAST)
                        fast_distances(d, nw, ne, sw, se, c, fr1);
                    else
                        exact_distances(d, nw, ne, sw, se, Sg[oh + lx], Sg[oh + lx + R], vu, vd, c, fr1, f2r1, N);
                    const Pick pk = select8<SEL>(d);
                    out_v[i] = S::bits(fmaf(pk.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c));
                    out_i[i] = pk.idx;
                }
            };
            if (s - R >= Y0 && s - R + CH <= yb) {  // uniform over the workgroup
                static_for<0, CH>([&](auto ic) { eval_row(ic); });
            } else {
                static_for<0, CH>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    if (s - R + i >= Y0 && s - R + i < yb) eval_row(ic);
                });
            }
        }
        out_s = s;
        pending = true;
    };

    for (int n = 0; n < nsteps; n += NRB) {
        static_for<0, NRB>([&](auto ph) {
            if (n + decltype(ph)::value < nsteps) step(ph, n + decltype(ph)::value);
        });
    }
    if (pending && own) store_step();
}

// Two fused sweeps on one work item (small radii): stage A runs the first
// sweep on the strip grown by R on each side (rows grown by R), reading the
// input from global memory; its rounded results are written straight into
// stage B's register ring as B's new input rows, from which stage B runs the
// second sweep on the strip itself.  Rows stage B needs above row 0 or below
// row H-1 are replicated from those rows (the clamp), so stage B sees exactly
// the clamp extension of the first sweep's output.  The region is TW + 4R
// columns wide; four barriers per step of CH rows of both sweeps (five in
// strips at an image edge).  LDS: CH blocks of four rows (A's P, the V rows
// both stages share, B's P, the H rows both share: A's evaluation may still
// read its P while B stages its own), one Q ring of L rows per stage and 2L
// floats for the edge columns.  Registers and LDS offsets follow
// the single-sweep item (rings unrolled over their period).  Every block and
// column anchor is a multiple of R, so the results are those of two
// single-sweep launches, bit for bit.
template <int DT, int R, int RW, int CH, bool SEL, int MODE>
__device__ __forceinline__ void fwd_stream2_item(const FwdLaunch &a, int t, float *lds) {
    using S = Storage<DT>;
    using T = typename S::T;
    static_assert(CH % R == 0, "a step is whole blocks of R rows");
    static_assert(RW % 64 == 0 && RW >= 5 * R, "region width");
    constexpr int M = CH / R, NRB = M + 1, L = R + CH, PITCH = RW + 1;
    constexpr int RS = 4 * PITCH + 29;      // staging block: PA, V, PB, H rows (stride 1 mod 32)
    float *const Sg = lds;
    float *const QA = lds + CH * RS;        // L rows (stage A ring)
    float *const QB = QA + L * PITCH;       // L rows (stage B ring)
    float *const Ex = QB + L * PITCH;       // 2L: ring rows of columns 0 and W - 1

    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int yb = min(H, Y0 + YC);
    const int ox = X0 - 2 * R;  // image column of region column 0
    const int x = ox + lx;

    // stage geometry: evaluated columns [xa, xb) and rows [ya, ye), fields
    // on columns [xa, xend) and rows up to yend
    struct Geo { int xa, xb, xend, ya, ye, yend, nb; };
    auto geo = [&](int xa, int xb, int ya, int ye) {
        Geo g;
        g.xa = xa; g.xb = xb; g.xend = xb + R;
        g.ya = ya; g.ye = ye; g.yend = ye + R;
        g.nb = (g.xend - xa + R - 1) / R;
        return g;
    };
    const Geo gA = geo(max(0, X0 - R), min(W, X0 + TW + R), max(0, Y0 - R), min(H, yb + R));
    const Geo gB = geo(X0, min(W, X0 + TW), Y0, yb);
    const bool ownA = x >= gA.xa && x < gA.xb, ownB = x >= gB.xa && x < gB.xb;
    const int nsteps = (yb + 2 * R - gA.ya + CH - 1) / CH;

    // rows up to the last one loaded or stored
    const ItemRows io = item_rows<T>(a, plane, max(0, gA.ya - R), min(H, gA.ya + nsteps * CH), SEL);
    BufRsrc selB = io.sel;
    if (SEL) {
        const size_t first = (size_t)plane * H * W + (size_t)io.row0 * W;
        const uint32_t n = (uint32_t)(min(H, gA.ya + nsteps * CH) - io.row0) * (uint32_t)W;
        selB = buf_rsrc(a.sel + a.sel_stride + first, n);
    }
    const int vld = clampi(x, 0, W - 1) * (int)sizeof(T);
    const int vst = x * (int)sizeof(T);

    // each stage's row-sum items, the same every step (as fwd_stream_item);
    // ib: the item's first LDS column relative to its row
    struct Items { int row[M], ib[M]; bool ok[M], full[M]; };
    auto items = [&](const Geo &g) {
        Items it;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = lx + k * RW;
            const int m = i / (R * g.nb), rem = i - m * (R * g.nb);
            const int b = rem / R;
            it.ok[k] = i < CH * g.nb;
            it.row[k] = m * R + (rem - b * R);
            const int x0 = g.xa + b * R;
            it.ib[k] = x0 - R - ox;
            it.full[k] = x0 + R <= g.xend;
        }
        return it;
    };
    const Items iA = items(gA), iB = items(gB);

    constexpr float fr1 = (float)(R + 1), f2r1 = (float)(2 * R + 1);
    constexpr float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    float PA[L], VA[L], PB[L], VB[L];  // physical rings of both stages
#pragma unroll
    for (int j = 0; j < R; ++j) {
        PA[j] = S::from_raw(S::load_raw(io.src, vld, io.ld_off(gA.ya - R + j)));
        VA[j] = PB[j] = VB[j] = 0.f;
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        PA[R + j] = S::load_raw(io.src, vld, io.ld_off(gA.ya + j));
        PB[R + j] = 0.f;
    }
    float outB[CH];
    int idxA[CH], idxB[CH];
    float hold = 0.f;  // stage A's row H - 1 (bottom chunks)
    int outB_s = 0;
    bool pending = false;
    auto store_prev = [&]() {
        if (!SEL && outB_s - R >= Y0 && outB_s - R + CH <= yb) {  // uniform: offsets step by a row
            int o = io.st_off(outB_s - R);
#pragma unroll
            for (int i = 0; i < CH; ++i, o += io.drow) S::store(io.dst, vst, o, outB[i]);
            return;
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int y = outB_s - R + i;  // stage B's rows of the previous step
            if (y >= Y0 && y < yb) {
                S::store(io.dst, vst, io.st_off(y), outB[i]);
                if (SEL) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)idxB[i], selB, x, io.sel_off(y), 0);
            }
            const int ya = outB_s + i;  // stage A's rows of the previous step
            if (SEL && ya >= Y0 && ya < yb)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)idxA[i], io.sel, x, io.sel_off(ya), 0);
        }
    };

    // V of the step's new rows into the ring, P of the rows evaluated this
    // step and the new V rows to LDS (P at staging row `prow` of each block)
    auto v_phase = [&](auto ph, float *P, float *V, int prow) {
        constexpr int PH = decltype(ph)::value;
        auto sl = [](int j) { return (j + PH * CH) % L; };
#pragma unroll
        for (int m = 0; m < M; ++m) {
            float v = P[sl(m * R)];
#pragma unroll
            for (int tt = 1; tt <= R; ++tt) v += P[sl(m * R + tt)];
            V[sl(R + m * R)] = v;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                v += P[sl(R + m * R + tt)] - P[sl(m * R + tt - 1)];
                V[sl(R + m * R + tt)] = v;
            }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            Sg[i * RS + prow * PITCH + lx] = P[sl(i)];
            Sg[i * RS + PITCH + lx] = V[sl(R + i)];
        }
    };
    // Q of rows [s, s + CH) into the ring, H of rows [s - R, s - R + CH);
    // the item reads P at staging row prow and V at row 1 of each block
    auto qh_phase = [&](auto ph, const Geo &g, const Items &it, int s0, float *Q, int prow) {
        constexpr int PH = decltype(ph)::value;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int i = it.row[k];
            if (!it.ok[k] || s0 + i >= g.yend) continue;
            const int ib = i * RS + it.ib[k];
            float v[2 * R], p[2 * R];
#pragma unroll
            for (int tt = 0; tt < 2 * R; ++tt) {
                p[tt] = Sg[ib + prow * PITCH + tt];
                v[tt] = Sg[ib + PITCH + tt];
            }
            const int qr = (PH * CH + R) % L + i;
            float *qrow_p = Q + (qr >= L ? qr - L : qr) * PITCH + it.ib[k] + R;
            float *hrow_p = Sg + ib + 3 * PITCH + R;
            constexpr bool HF = MODE != MODE_FAST;
            float q = v[0], h = p[0];
#pragma unroll
            for (int tt = 1; tt <= R; ++tt) {
                q += v[tt];
                if (HF) h += p[tt];
            }
            qrow_p[0] = q;
            if (HF) hrow_p[0] = h;
            if (it.full[k]) {
#pragma unroll
                for (int tt = 1; tt < R; ++tt) {
                    q += v[R + tt] - v[tt - 1];
                    qrow_p[tt] = q;
                    if (HF) {
                        h += p[R + tt] - p[tt - 1];
                        hrow_p[tt] = h;
                    }
                }
            } else {
                const int x0 = it.ib[k] + R + ox;
#pragma unroll
                for (int tt = 1; tt < R; ++tt) {
                    if (x0 + tt < g.xend) {
                        q += v[R + tt] - v[tt - 1];
                        qrow_p[tt] = q;
                        if (HF) {
                            h += p[R + tt] - p[tt - 1];
                            hrow_p[tt] = h;
                        }
                    }
                }
            }
        }
    };
    // rows [s - R, s - R + CH) ∩ [ya, ye) of this lane's column; fn(i, value,
    // index) with i an integral constant
    auto eval_phase = [&](auto ph, const Geo &g, int s0, const float *Q, const float *V, int prow, auto &&fn) {
        constexpr int PH = decltype(ph)::value;
        auto sl = [](int j) { return (j + PH * CH) % L; };
        auto qrow = [](int j) { return (PH * CH + R + j) % L; };
        static_for<0, CH>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int y = s0 - R + i;
            if (y < g.ya || y >= g.ye) return;  // uniform over the workgroup
            constexpr int ou = qrow(i - R) * PITCH, od = qrow(i) * PITCH;
            const int op = i * RS + prow * PITCH, oh = i * RS + 3 * PITCH;
            const float c = Sg[op + lx];
            const float nw = Q[ou + lx], ne = Q[ou + lx + R], sw = Q[od + lx], se = Q[od + lx + R];
            const float vu = V[sl(i)], vd = V[sl(i + R)];
            if constexpr (MODE == MODE_BOX) {
                fn(ic, S::round(box_sum(nw, ne, sw, se, Sg[oh + lx], Sg[oh + lx + R], vu, vd, c) * inv_box), 0);
            } else {
                float d[8];
                if constexpr (MODE == MODE_FAST)
                    fast_distances(d, nw, ne, sw, se, c, fr1);
                else
                    exact_distances(d, nw, ne, sw, se, Sg[oh + lx], Sg[oh + lx + R], vu, vd, c, fr1, f2r1, N);
                const Pick pk = select8<SEL>(d);
                fn(ic, S::round(fmaf(pk.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c)), pk.idx);
            }
        });
    };

    auto step = [&](auto ph, int n) {
        constexpr int PH = decltype(ph)::value;
        auto sl = [](int j) { return (j + PH * CH) % L; };
        const int sA = gA.ya + n * CH, sB = sA - R;
        // stage A: the first sweep from the input
#pragma unroll
        for (int j = R; j < L; ++j) PA[sl(j)] = S::from_raw(PA[sl(j)]);
        v_phase(ph, PA, VA, 0);
        if (pending && ownB) store_prev();
        if (n + 1 < nsteps) {
            if (sA + CH >= 0 && sA + 2 * CH <= H) {  // uniform: no clamped row
                int o = io.ld_off(sA + CH);
#pragma unroll
                for (int i = 0; i < CH; ++i, o += io.srow) PA[sl(i)] = S::load_raw(io.src, vld, o);
            } else {
#pragma unroll
                for (int i = 0; i < CH; ++i) PA[sl(i)] = S::load_raw(io.src, vld, io.ld_off(sA + CH + i));
            }
        }
        __syncthreads();
        qh_phase(ph, gA, iA, sA, QA, 0);
        __syncthreads();
        // stage A's results are stage B's new rows [sB, sB + CH) (logical
        // ring rows j <-> image rows sB - R + j); rows stage B reads above
        // row 0 repeat row 0 (set when row 0 is produced: they are the ring
        // rows below it then), rows below row H - 1 repeat row H - 1
        if (ownA) {
            eval_phase(ph, gA, sA, QA, VA, 0, [&](auto ic, float u, int m) {
                constexpr int i = decltype(ic)::value;
                PB[sl(R + i)] = u;
                idxA[i] = m;
                const int y = sA - R + i;
                if (y == 0) static_for<0, R + i>([&](auto jc) { PB[sl(decltype(jc)::value)] = u; });
                if (y == H - 1) hold = u;
            });
            static_for<0, CH>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if (sA - R + i >= H) PB[sl(R + i)] = hold;
            });
        }
        // Stage B's row sums read columns [X0 - R, min(W, X0 + TW) + R); at
        // an image edge the lanes outside the image take column 0 or W - 1
        // (the clamp), which stage A computed in another lane.
        if (X0 == 0 || X0 + TW + R > W) {  // uniform
            if (x == 0) static_for<0, L>([&](auto jc) { Ex[decltype(jc)::value] = PB[sl(decltype(jc)::value)]; });
            if (x == W - 1) static_for<0, L>([&](auto jc) { Ex[L + decltype(jc)::value] = PB[sl(decltype(jc)::value)]; });
            __syncthreads();
            if (x < 0) static_for<0, L>([&](auto jc) { PB[sl(decltype(jc)::value)] = Ex[decltype(jc)::value]; });
            if (x >= W) static_for<0, L>([&](auto jc) { PB[sl(decltype(jc)::value)] = Ex[L + decltype(jc)::value]; });
        }
        // stage B: the second sweep
        v_phase(ph, PB, VB, 2);
        __syncthreads();
        qh_phase(ph, gB, iB, sB, QB, 2);
        __syncthreads();
        if (ownB)
            eval_phase(ph, gB, sB, QB, VB, 2, [&](auto ic, float u, int m) {
                constexpr int i = decltype(ic)::value;
                outB[i] = u;
                idxB[i] = m;
            });
        outB_s = sB;
        pending = true;
    };

    for (int n = 0; n < nsteps; n += NRB) {
        static_for<0, NRB>([&](auto ph) {
            if (n + decltype(ph)::value < nsteps) step(ph, n + decltype(ph)::value);
        });
    }
    if (pending && ownB) store_prev();
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
    // a work item addresses its rows through 32-bit offsets from its first row
    const long long row_bytes = (long long)a.W * (DT == DT_F32 ? 4 : 2);
    auto fits = [&](long long rows) { return (rows + 4 * R + 2 * CH) * row_bytes < (1LL << 31); };
    if (a.th > 0 && !fits(a.th)) return hipErrorInvalidValue;
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
        constexpr int RQ = stream_row_quantum(R);
        int rows = (a.H + per_strip - 1) / per_strip;
        rows = std::max(RQ, (rows + RQ - 1) / RQ * RQ);
        while (rows > RQ && !fits(rows)) rows = std::max(RQ, rows / 2 / RQ * RQ);
        if (!fits(rows)) return hipErrorInvalidValue;
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
