// Forward kernels of the one-sided box filter (Alg. 2), gfx950.
//
// One workgroup owns a TW x TH output tile of one plane and runs k Jacobi
// sweeps on it without leaving LDS (temporal blocking).  It loads the tile
// plus a k*r halo once (clamped to the image), and sweep j (0-based) updates
// the tile grown by (k-1-j)*r on each side, clipped to the image.  Reads of
// the replicate extension are clamped to image coordinates; a clamped read
// never leaves the region the previous sweep produced.
//
// The eight window sums come from three separable running-sum fields
// (O(1) in r per pixel, Sec. III-D), defined on the clamp extension P:
//   V(x,y) = sum_{y'=y-r..y} P(x,y')     upward (r+1)-tall column sum
//   Q(x,y) = sum_{x'=x-r..x} V(x',y)     north-west quadrant sum ending at (x,y)
//   H(x,y) = sum_{x'=x-r..x} P(x',y)     leftward (r+1)-wide row sum
// so that NW = Q(x,y), NE = Q(x+r,y), SW = Q(x,y+r), SE = Q(x+r,y+r),
//   L = NW + SW - H(x,y), R = NE + SE - H(x+r,y),
//   U = NW + NE - V(x,y), D = SW + SE - V(x,y+r)
// (each half is two quadrants minus the shared centre row or column).
//
// Position-determinism: every running sum restarts at image coordinates that
// are multiples of r (a direct sum of r+1 terms in a fixed order, then at most
// r-1 slide steps), tiles are multiples of r, and every fused sweep's region
// starts on such a multiple.  The FP32 operations that produce a pixel's value
// therefore depend only on its position, never on the tile, the fusion depth
// or the launch shape: fused launches, single-sweep launches and the batched
// kernel give bit-identical results and selection maps.
//
// Phase A fills V down columns, phase B fills Q and H along rows, phase C
// evaluates the eight scaled distances and the tie-ordered argmin per pixel.
// Fields live in LDS as FP32; the kernel is bound by VALU and LDS throughput,
// not MFMA (there is no dense contraction on this path).
#pragma once
#include "osbf_device.h"
#include "osbf_internal.h"

namespace osbf {

enum : int { MODE_EXACT = 0, MODE_FAST = 1, MODE_BOX = 2 };

// Sum of the full (2r+1)^2 box from the same fields: the four quadrants
// cover it with the centre row segments [x-r,x] and [x,x+r] and the centre
// column segments counted twice and the centre pixel four times.
__device__ __forceinline__ float box_sum(float nw, float ne, float sw, float se, float hl, float hr,
                                         float vu, float vd, float c) {
    return ((nw + ne) + (sw + se)) - ((hl + hr) + (vu + vd)) + c;
}

// Signed scaled differences of the exact filter (Alg. 2): N times
// (mean_i - c) for the windows R, L, D, U, SE, SW, NE, NW, from the four
// quadrant sums, the row sums H at x and x+r and the column sums V at y and
// y+r (each half is two quadrants minus their shared row or column).
__device__ __forceinline__ void exact_distances(float d[8], float nw, float ne, float sw, float se,
                                                float hl, float hr, float vu, float vd, float c,
                                                float fr1, float f2r1, float N) {
    const float sR = ne + se - hr;
    const float sL = nw + sw - hl;
    const float sD = sw + se - vd;
    const float sU = nw + ne - vu;
    const float nc = -N * c;
    d[0] = fmaf(fr1, sR, nc);
    d[1] = fmaf(fr1, sL, nc);
    d[2] = fmaf(fr1, sD, nc);
    d[3] = fmaf(fr1, sU, nc);
    d[4] = fmaf(f2r1, se, nc);
    d[5] = fmaf(f2r1, sw, nc);
    d[6] = fmaf(f2r1, ne, nc);
    d[7] = fmaf(f2r1, nw, nc);
}

// Signed scaled differences of the fast approximation (Alg. 3): 2 (r+1)^2
// times (candidate - c), where each half is the average of its two
// quadrants (eq:app) and the quadrants are the quadrant means themselves.
__device__ __forceinline__ void fast_distances(float d[8], float nw, float ne, float sw, float se,
                                               float c, float fr1) {
    const float nc = -2.f * fr1 * fr1 * c;
    d[0] = (ne + se) + nc;
    d[1] = (nw + sw) + nc;
    d[2] = (sw + se) + nc;
    d[3] = (nw + ne) + nc;
    d[4] = fmaf(2.f, se, nc);
    d[5] = fmaf(2.f, sw, nc);
    d[6] = fmaf(2.f, ne, nc);
    d[7] = fmaf(2.f, nw, nc);
}

template <bool CL>
__device__ __forceinline__ int cidx(int v, int hi) {
    return CL ? min(max(v, 0), hi) : v;
}

// Phase A: V on columns [vx0, vx1), rows [ya, yend), blocks of r rows
// anchored at multiples of r.  Pi, Vi index image coordinates.
template <int R, bool CL>
__device__ __forceinline__ void phase_v(const float *Pi, float *Vi, int pitch, int r, int H,
                                        int vx0, int vx1, int ya, int yend, int tx, int ty) {
    const int nblk = (yend - ya + r - 1) / r;
    for (int b = ty; b < nblk; b += 4) {
        const int y0 = ya + b * r;
        const int y1 = min(y0 + r, yend);
        for (int x = vx0 + tx; x < vx1; x += 64) {
            const float *pc = Pi + x;
            float *vc = Vi + x;
            float v = pc[cidx<CL>(y0 - r, H - 1) * pitch];
            if (R > 0) {
#pragma unroll
                for (int t = 1; t <= R; ++t) v += pc[cidx<CL>(y0 - R + t, H - 1) * pitch];
                vc[y0 * pitch] = v;
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    const int y = y0 + t;
                    if (y < y1) {
                        v += pc[cidx<CL>(y, H - 1) * pitch] - pc[cidx<CL>(y - R - 1, H - 1) * pitch];
                        vc[y * pitch] = v;
                    }
                }
            } else {
                for (int t = 1; t <= r; ++t) v += pc[cidx<CL>(y0 - r + t, H - 1) * pitch];
                vc[y0 * pitch] = v;
                for (int y = y0 + 1; y < y1; ++y) {
                    v += pc[cidx<CL>(y, H - 1) * pitch] - pc[cidx<CL>(y - r - 1, H - 1) * pitch];
                    vc[y * pitch] = v;
                }
            }
        }
    }
}

// Phase B: Q on columns [xa, xend), rows [ya, yq); H on the same columns,
// rows [ya, yh).  Blocks of r columns anchored at multiples of r.
template <int R, bool CL, int MODE = 0>
__device__ __forceinline__ void phase_qh(const float *Pi, const float *Vi, float *Qi, float *Hi,
                                         int pitch, int r, int W, int xa, int xend, int ya, int yq,
                                         int yh, int tx, int ty) {
    const int nblk = (xend - xa + r - 1) / r;
    const int nrow = yq - ya;
    for (int b = ty; b < nblk; b += 4) {
        const int x0 = xa + b * r;
        const int x1 = min(x0 + r, xend);
        for (int rr = tx; rr < nrow; rr += 64) {
            const int y = ya + rr;
            const bool doH = MODE != MODE_FAST && y < yh;
            const float *vr = Vi + y * pitch;
            const float *pr = Pi + y * pitch;
            float *qr = Qi + y * pitch;
            float *hr = Hi + y * pitch;
            const int c0 = cidx<CL>(x0 - r, W - 1);
            float q = vr[c0], h = doH ? pr[c0] : 0.f;
            if (R > 0) {
#pragma unroll
                for (int t = 1; t <= R; ++t) {
                    const int cx = cidx<CL>(x0 - R + t, W - 1);
                    q += vr[cx];
                    if (doH) h += pr[cx];
                }
                qr[x0] = q;
                if (doH) hr[x0] = h;
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    const int x = x0 + t;
                    if (x < x1) {
                        const int cn = cidx<CL>(x, W - 1), co = cidx<CL>(x - R - 1, W - 1);
                        q += vr[cn] - vr[co];
                        qr[x] = q;
                        if (doH) {
                            h += pr[cn] - pr[co];
                            hr[x] = h;
                        }
                    }
                }
            } else {
                for (int t = 1; t <= r; ++t) {
                    const int cx = cidx<CL>(x0 - r + t, W - 1);
                    q += vr[cx];
                    if (doH) h += pr[cx];
                }
                qr[x0] = q;
                if (doH) hr[x0] = h;
                for (int x = x0 + 1; x < x1; ++x) {
                    const int cn = cidx<CL>(x, W - 1), co = cidx<CL>(x - r - 1, W - 1);
                    q += vr[cn] - vr[co];
                    qr[x] = q;
                    if (doH) {
                        h += pr[cn] - pr[co];
                        hr[x] = h;
                    }
                }
            }
        }
    }
}

// k fused sweeps on one tile.  `lds` holds four arrays of a.arr floats.
// MODE: MODE_EXACT (Alg. 2), MODE_FAST (the approximation of Alg. 3: quadrant
// means only, halves as pair averages, no H field) or MODE_BOX (the classical
// (2r+1)^2 box mean the paper times its filter against).
template <int DT, int R, bool SEL, int MODE = 0>
__device__ __forceinline__ void fwd_tile(const FwdLaunch &a, int tile_x, int tile_y, int plane,
                                         float *lds) {
    using S = Storage<DT>;
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int r = R > 0 ? R : a.r;
    const int H = a.H, W = a.W, k = a.k, TW = a.tw, TH = a.th;
    const int ext = k * r;
    const int pitch = a.pitch;
    const int X0 = tile_x * TW, Y0 = tile_y * TH;
    const int ox = X0 - ext, oy = Y0 - ext;  // image coords of LDS (0,0)
    // image-coordinate views of the four LDS arrays
    const long shift = -(long)oy * pitch - ox;
    float *Pi = lds + shift;
    float *Vi = lds + a.arr + shift;
    float *Qi = lds + 2 * a.arr + shift;
    float *Hi = lds + 3 * a.arr + shift;
    const size_t plane_off = (size_t)plane * H * W;
    const typename S::T *src = (const typename S::T *)a.src + plane_off;
    const bool interior = (X0 - ext >= 0) && (Y0 - ext >= 0) && (X0 + TW + ext <= W) &&
                          (Y0 + TH + ext <= H);

    // Clamped load of the tile plus halo.
    {
        const int x0 = max(0, X0 - ext), x1 = min(W, X0 + TW + ext);
        const int y0 = max(0, Y0 - ext), y1 = min(H, Y0 + TH + ext);
        for (int y = y0 + ty; y < y1; y += 4) {
            float *prow = Pi + y * pitch;
            const size_t g = (size_t)y * W;
            for (int x = x0 + tx; x < x1; x += 64) prow[x] = S::load(src, g + x);
        }
    }
    __syncthreads();

    const float fr1 = (float)(r + 1), f2r1 = (float)(2 * r + 1);
    const float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    for (int j = 0; j < k; ++j) {
        const int e = (k - 1 - j) * r;
        const int xa = max(0, X0 - e), xb = min(W, X0 + TW + e);
        const int ya = max(0, Y0 - e), yb = min(H, Y0 + TH + e);

        wave_priority<1>();  // phases A and B gate the barriers; C fills in
        if (interior)
            phase_v<R, false>(Pi, Vi, pitch, r, H, xa - r, xb + r, ya, yb + r, tx, ty);
        else
            phase_v<R, true>(Pi, Vi, pitch, r, H, max(0, xa - r), min(W, xb + r), ya, yb + r, tx, ty);
        __syncthreads();
        wave_priority<2>();
        if (interior)
            phase_qh<R, false, MODE>(Pi, Vi, Qi, Hi, pitch, r, W, xa, xb + r, ya, yb + r, yb, tx, ty);
        else
            phase_qh<R, true, MODE>(Pi, Vi, Qi, Hi, pitch, r, W, xa, xb + r, ya, yb + r, yb, tx, ty);
        wave_priority<0>();
        __syncthreads();

        // Phase C: selection and update on [xa, xb) x [ya, yb).
        const bool last = (j == k - 1);
        uint8_t *sel = SEL ? a.sel + (size_t)j * a.sel_stride + plane_off : nullptr;
        typename S::T *dst = (typename S::T *)a.dst + plane_off;
        const int rp = r * pitch;
        for (int y = ya + ty; y < yb; y += 4) {
            for (int x = xa + tx; x < xb; x += 64) {
                const int o = y * pitch + x, od = o + rp;
                const float c = Pi[o];
                const float nw = Qi[o], ne = Qi[o + r], sw = Qi[od], se = Qi[od + r];
                float u;
                Pick p{0.f, 0};
                if constexpr (MODE == MODE_BOX) {
                    u = S::round(box_sum(nw, ne, sw, se, Hi[o], Hi[o + r], Vi[o], Vi[od], c) * inv_box);
                } else {
                    float d[8];
                    if constexpr (MODE == MODE_FAST)
                        fast_distances(d, nw, ne, sw, se, c, fr1);
                    else
                        exact_distances(d, nw, ne, sw, se, Hi[o], Hi[o + r], Vi[o], Vi[od], c, fr1, f2r1, N);
                    p = select8<SEL>(d);
                    u = S::round(fmaf(p.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c));
                }
                if (SEL) {
                    const bool core = (x >= X0) && (x < X0 + TW) && (y >= Y0) && (y < Y0 + TH);
                    if (core) sel[(size_t)y * W + x] = (uint8_t)p.idx;
                }
                if (last)
                    dst[(size_t)y * W + x] = S::pack(u);
                else
                    Pi[o] = u;
            }
        }
        if (!last) __syncthreads();
    }
}

template <int DT, int R, bool SEL, int MODE = 0>
__global__ __launch_bounds__(256) void fwd_tile_kernel(FwdLaunch a) {
    extern __shared__ float lds[];
    const int ntiles = a.tiles_x * a.tiles_y;
    const int total = ntiles * a.planes;
    const int t = xcd_remap(blockIdx.x, total);
    const int plane = t / ntiles, tile = t - plane * ntiles;
    fwd_tile<DT, R, SEL, MODE>(a, tile % a.tiles_x, tile / a.tiles_x, plane, lds);
}

// Phase A of the fixed-geometry kernel: V on columns [max(0,xa-R),
// min(W,xb+R)), rows [ya, yb+R), in blocks of R rows anchored at multiples of
// R.  Each lane owns one region column; a block's 2R input rows are read once.
template <int R, int RW, int RH, int NT, bool CL>
__device__ __forceinline__ void fixed_phase_v(const float *P, float *V, int lx, int ly, int ox,
                                              int oy, int H, int W, int xa, int xb, int ya, int yb) {
    constexpr int PITCH = RW + 1;
    constexpr int NY = NT / RW;
    const int x = ox + lx;
    if (x < max(0, xa - R) || x >= min(W, xb + R)) return;
    const int yend = yb + R;
    const int nblk = (yend - ya + R - 1) / R;
    for (int b = ly; b < nblk; b += NY) {
        const int y0 = ya + b * R;
        float p[2 * R];
        if (!CL) {
            const float *pc = P + (y0 - R - oy) * PITCH + lx;
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) p[t] = pc[t * PITCH];
        } else {
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) p[t] = P[(min(max(y0 - R + t, 0), H - 1) - oy) * PITCH + lx];
        }
        float *vc = V + (y0 - oy) * PITCH + lx;
        float v = p[0];
#pragma unroll
        for (int t = 1; t <= R; ++t) v += p[t];
        vc[0] = v;
        if (y0 + R <= yend) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                v += p[R + t] - p[t - 1];
                vc[t * PITCH] = v;
            }
        } else {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                if (y0 + t < yend) {
                    v += p[R + t] - p[t - 1];
                    vc[t * PITCH] = v;
                }
            }
        }
    }
}

// First sweep's phase A fused with the tile load: each lane loads, for every
// block of R rows its wave owns, the block's 2R input rows of its column
// straight from global memory (rows clamped into the image; all loads issued
// before the first wait), forms V in registers, and writes the block's own P
// and V rows to LDS.  No barrier is needed between load and phase A, and the
// FP32 operations are those of fixed_phase_v.
template <int DT, int R, int RW, int RH, int NT>
__device__ __forceinline__ void fixed_load_phase_v(const typename Storage<DT>::T *src, float *P, float *V,
                                                   int lx, int ly, int ox, int oy, int H, int W, int xa,
                                                   int xb, int ya, int yb) {
    using S = Storage<DT>;
    constexpr int PITCH = RW + 1;
    constexpr int NY = NT / RW;
    constexpr int MB = ((RH - 1) / R + NY - 1) / NY;  // blocks per wave, at most
    const int x = ox + lx;
    if (x < max(0, xa - R) || x >= min(W, xb + R)) return;
    const int yend = yb + R;
    const int nblk = (yend - ya + R - 1) / R;
    typename S::T raw[MB][2 * R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int b = ly + i * NY;
        if (b < nblk) {
            const int y0 = ya + b * R;
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) raw[i][t] = src[(size_t)min(max(y0 - R + t, 0), H - 1) * W + x];
        }
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int b = ly + i * NY;
        if (b >= nblk) break;
        const int y0 = ya + b * R;
        float p[2 * R];
#pragma unroll
        for (int t = 0; t < 2 * R; ++t) p[t] = S::cvt(raw[i][t]);
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int y = y0 + t;
            if (y < yend && y < H) P[(y - oy) * PITCH + lx] = p[R + t];
        }
        float *vc = V + (y0 - oy) * PITCH + lx;
        float v = p[0];
#pragma unroll
        for (int t = 1; t <= R; ++t) v += p[t];
        vc[0] = v;
        if (y0 + R <= yend) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                v += p[R + t] - p[t - 1];
                vc[t * PITCH] = v;
            }
        } else {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                if (y0 + t < yend) {
                    v += p[R + t] - p[t - 1];
                    vc[t * PITCH] = v;
                }
            }
        }
    }
}

// Phase B of the fixed-geometry kernel: Q on columns [xa, xb+R), rows
// [ya, yb+R); H on the same columns, rows [ya, yb).  One lane per region row.
template <int R, int RW, int RH, int NT, bool CL, int MODE = 0>
__device__ __forceinline__ void fixed_phase_qh(const float *P, const float *V, float *Q, float *Hs,
                                               int lr, int lb, int ox, int oy, int W, int xa,
                                               int xb, int ya, int yb) {
    constexpr int PITCH = RW + 1;
    constexpr int NB = NT / 64;  // lane groups over column blocks
    const int y = oy + lr;
    if (lr >= RH || y < ya || y >= yb + R) return;
    const bool doH = MODE != MODE_FAST && y < yb;
    const int xend = xb + R;
    const int nblk = (xend - xa + R - 1) / R;
    for (int b = lb; b < nblk; b += NB) {
        const int x0 = xa + b * R;
        float v[2 * R], p[2 * R];
        if (!CL) {
            const int o = lr * PITCH + (x0 - R - ox);
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) {
                v[t] = V[o + t];
                p[t] = P[o + t];
            }
        } else {
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) {
                const int o = lr * PITCH + (min(max(x0 - R + t, 0), W - 1) - ox);
                v[t] = V[o];
                p[t] = P[o];
            }
        }
        float *qr = Q + lr * PITCH + (x0 - ox);
        float *hr = Hs + lr * PITCH + (x0 - ox);
        float q = v[0], h = p[0];
#pragma unroll
        for (int t = 1; t <= R; ++t) {
            q += v[t];
            h += p[t];
        }
        qr[0] = q;
        if (doH) hr[0] = h;
        if (x0 + R <= xend) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                q += v[R + t] - v[t - 1];
                h += p[R + t] - p[t - 1];
                qr[t] = q;
                if (doH) hr[t] = h;
            }
        } else {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                if (x0 + t < xend) {
                    q += v[R + t] - v[t - 1];
                    h += p[R + t] - p[t - 1];
                    qr[t] = q;
                    if (doH) hr[t] = h;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fixed-geometry kernel for the common radii.  The LDS region is RW x RH
// pixels (halo included) with a compile-time pitch, so every LDS access is an
// immediate offset from one base address; one wave spans a region row.  The
// arithmetic is the same sequence of FP32 operations as fwd_tile (same block
// anchors, same summation order), so both kernels give identical bits.
template <int DT, int R, int RW, int RH, int NT, bool SEL, int MODE = 0>
__device__ __forceinline__ void fwd_fixed(const FwdLaunch &a, int tile_x, int tile_y, int plane,
                                          float *lds) {
    using S = Storage<DT>;
    constexpr int PITCH = RW + 1;
    constexpr int ARR = RH * PITCH;
    constexpr int NY = NT / RW;  // region rows handled at once
    static_assert(RW == 64 || RW == 128, "region width");
    static_assert(NT % RW == 0 && NT % 64 == 0, "thread count");
    static_assert(RH <= 64, "phase B maps one lane per region row");
    float *const P = lds;
    float *const V = lds + ARR;
    float *const Q = lds + 2 * ARR;
    float *const Hs = lds + 3 * ARR;
    const int tid = threadIdx.x;
    // phase A / C: lane = region column; phase B: lane = region row.  The
    // wave-level indices are uniform, so loop control stays on the SALU.
    const int lx = tid % RW, ly = __builtin_amdgcn_readfirstlane(tid / RW);
    const int lr = tid & 63, lb = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int H = a.H, W = a.W, k = a.k, TW = a.tw, TH = a.th;
    const int ext = k * R;
    const int X0 = tile_x * TW, Y0 = tile_y * TH;
    const int ox = X0 - ext, oy = Y0 - ext;  // image coords of LDS (0,0)
    const size_t plane_off = (size_t)plane * H * W;
    const typename S::T *src = (const typename S::T *)a.src + plane_off;
    const bool interior = (X0 - ext >= 0) && (Y0 - ext >= 0) && (X0 + TW + ext <= W) &&
                          (Y0 + TH + ext <= H);

    constexpr float fr1 = (float)(R + 1), f2r1 = (float)(2 * R + 1);
    constexpr float N = fr1 * fr1 * f2r1;
    const float invN = 1.0f / N;
    const float inv_box = 1.0f / (f2r1 * f2r1);

    for (int j = 0; j < k; ++j) {
        const int e = (k - 1 - j) * R;
        const int xa = max(0, X0 - e), xb = min(W, X0 + TW + e);
        const int ya = max(0, Y0 - e), yb = min(H, Y0 + TH + e);

        wave_priority<1>();  // phases A and B gate the barriers; C fills in (as the streaming kernel)
        if (j == 0)  // the load of the tile + halo, fused with the first phase A
            fixed_load_phase_v<DT, R, RW, RH, NT>(src, P, V, lx, ly, ox, oy, H, W, xa, xb, ya, yb);
        else if (interior)
            fixed_phase_v<R, RW, RH, NT, false>(P, V, lx, ly, ox, oy, H, W, xa, xb, ya, yb);
        else
            fixed_phase_v<R, RW, RH, NT, true>(P, V, lx, ly, ox, oy, H, W, xa, xb, ya, yb);
        __syncthreads();
        wave_priority<2>();
        if (interior)
            fixed_phase_qh<R, RW, RH, NT, false, MODE>(P, V, Q, Hs, lr, lb, ox, oy, W, xa, xb, ya, yb);
        else
            fixed_phase_qh<R, RW, RH, NT, true, MODE>(P, V, Q, Hs, lr, lb, ox, oy, W, xa, xb, ya, yb);
        wave_priority<0>();
        __syncthreads();

        // Phase C: selection and update on [xa, xb) x [ya, yb).
        {
            const bool last = (j == k - 1);
            const int x = ox + lx;
            if (x >= xa && x < xb) {
                uint8_t *sel = SEL ? a.sel + (size_t)j * a.sel_stride + plane_off : nullptr;
                typename S::T *dst = (typename S::T *)a.dst + plane_off;
                const bool core_x = x >= X0 && x < X0 + TW;
                auto update = [&](int y, float &u, int &idx) {
                    const int o = (y - oy) * PITCH + lx;
                    constexpr int RD = R * PITCH;
                    const float c = P[o];
                    const float nw = Q[o], ne = Q[o + R], sw = Q[o + RD], se = Q[o + RD + R];
                    if constexpr (MODE == MODE_BOX) {
                        u = S::round(box_sum(nw, ne, sw, se, Hs[o], Hs[o + R], V[o], V[o + RD], c) * inv_box);
                        idx = 0;
                    } else {
                        float d[8];
                        if constexpr (MODE == MODE_FAST)
                            fast_distances(d, nw, ne, sw, se, c, fr1);
                        else
                            exact_distances(d, nw, ne, sw, se, Hs[o], Hs[o + R], V[o], V[o + RD], c, fr1, f2r1, N);
                        const Pick pk = select8<SEL>(d);
                        u = S::round(fmaf(pk.d, MODE == MODE_FAST ? 0.5f / (fr1 * fr1) : invN, c));
                        idx = pk.idx;
                    }
                    return o;
                };
                if (last) {
                    for (int y = ya + ly; y < yb; y += NY) {
                        float u;
                        int idx;
                        update(y, u, idx);
                        if (SEL && core_x && y >= Y0 && y < Y0 + TH) sel[(size_t)y * W + x] = (uint8_t)idx;
                        dst[(size_t)y * W + x] = S::pack(u);
                    }
                } else {
                    for (int y = ya + ly; y < yb; y += NY) {
                        float u;
                        int idx;
                        const int o = update(y, u, idx);
                        if (SEL && core_x && y >= Y0 && y < Y0 + TH) sel[(size_t)y * W + x] = (uint8_t)idx;
                        P[o] = u;
                    }
                }
            }
            if (!last) __syncthreads();
        }
    }
}

template <int DT, int R, int RW, int RH, int NT, bool SEL, int MODE = 0>
__global__ __launch_bounds__(NT) void fwd_fixed_kernel(FwdLaunch a) {
    extern __shared__ float lds[];
    const int ntiles = a.tiles_x * a.tiles_y;
    const int total = ntiles * a.planes;
    const int t = xcd_remap(blockIdx.x, total);
    const int plane = t / ntiles, tile = t - plane * ntiles;
    fwd_fixed<DT, R, RW, RH, NT, SEL, MODE>(a, tile % a.tiles_x, tile / a.tiles_x, plane, lds);
}

}  // namespace osbf
