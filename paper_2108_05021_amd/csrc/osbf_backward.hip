// Adjoint of one sweep of the one-sided box filter, gfx950.
//
// With the selection map m(p) of a forward sweep held fixed, the sweep is the
// linear map  U'(p) = (1/n_m) * sum_{q in W_m(p)} U(clamp(q)).  Its transpose
// sends an upstream gradient G' to
//     G(s) = sum_{q : clamp(q) = s} Gpad(q),
//     Gpad(q) = sum_p gv(p) [q in W_m(p)(p)],   gv(p) = G'(p) / n_m(p),
// where q runs over the image grown by r (the replicate extension) and the
// outer sum folds that halo back onto the edge pixels (adjoint of the clamp).
//
// Each window is X_m(px) x Y_m(py) with X, Y one-sided or centred ranges, so
// q in W_m(p) splits into px in the reflected X range of qx and py in the
// reflected Y range of qy.  Grouping the eight windows by reflected X range:
//   VL = Vup[F_R + F_SE] + Vdown[F_R + F_NE] - F_R      (X range [qx-r, qx])
//   VR = Vup[F_L + F_SW] + Vdown[F_L + F_NW] - F_L      (X range [qx, qx+r])
//   VF = Vup[F_D] + Vdown[F_U]                          (X range [qx-r, qx+r])
//   Gpad = Hl[VL + VF] + Hr[VR + VF] - VF
// with F_m = gv [m(p) = m], Vup/Vdown the (r+1)-tall sums ending/starting at
// the row, Hl/Hr the (r+1)-wide sums ending/starting at the column.  It is a
// gather: every output is written by exactly one workgroup, no atomics.
//
// Running sums restart at image positions that are multiples of r (direct
// sum, then slides), as in the forward kernels, so results do not depend on
// the tile shape.
#include <algorithm>

#include "osbf_device.h"
#include "osbf_internal.h"

namespace osbf {

// Membership of window m in the eight masked fields, as bit masks over m
// (R=0 L=1 D=2 U=3 SE=4 SW=5 NE=6 NW=7).
enum : unsigned {
    M_C1 = 0x11,  // R + SE   (up,   into VL)
    M_C2 = 0x41,  // R + NE   (down, into VL)
    M_C3 = 0x22,  // L + SW   (up,   into VR)
    M_C4 = 0x82,  // L + NW   (down, into VR)
    M_FR = 0x01, M_FL = 0x02, M_FD = 0x04, M_FU = 0x08
};

// gv if window `s` belongs to mask M, else 0 (bit-exact select).
__device__ __forceinline__ float pick(unsigned M, int s, float gv) {
    const int all = __builtin_amdgcn_sbfe((int)M, s, 1);  // 0 or -1
    return __int_as_float(__float_as_int(gv) & all);
}

template <bool CL>
__device__ __forceinline__ int bidx(int v, int lo, int hi) {
    return CL ? min(max(v, lo), hi) : v;
}

__global__ __launch_bounds__(256) void adjoint_kernel(BwdLaunch a) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int r = a.r, H = a.H, W = a.W, TW = a.tw, TH = a.th;
    const int pitch = a.pitch;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int t = blockIdx.x;
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int X0 = (tile % a.tiles_x) * TW, Y0 = (tile / a.tiles_x) * TH;
    const int ox = X0 - 2 * r, oy = Y0 - 2 * r;
    const long shift = -(long)oy * pitch - ox;
    float *GV = lds + shift;                 // gv, later Gpad
    int *SL = (int *)(lds + a.arr) + shift;  // selection
    float *HL = lds + 2 * a.arr + shift;
    float *HR = lds + 3 * a.arr + shift;
    float *VF = lds + 4 * a.arr + shift;
    const size_t plane_off = (size_t)plane * H * W;
    const float *gn = a.gnext + plane_off;
    const uint8_t *sl = a.sel + plane_off;

    // q region: the tile, grown by r beyond every image edge it touches
    const int qx0 = X0 == 0 ? -r : X0, qx1 = X0 + TW >= W ? W + r : X0 + TW;
    const int qy0 = Y0 == 0 ? -r : Y0, qy1 = Y0 + TH >= H ? H + r : Y0 + TH;
    const float inv_h = 1.0f / (float)((r + 1) * (2 * r + 1));
    const float inv_q = 1.0f / (float)((r + 1) * (r + 1));

    // Phase 0: gv and selection on the F region (zero outside the image).
    for (int y = qy0 - r + ty; y < qy1 + r; y += 4) {
        const bool yin = y >= 0 && y < H;
        for (int x = qx0 - r + tx; x < qx1 + r; x += 64) {
            const int o = y * pitch + x;
            if (yin && x >= 0 && x < W) {
                const size_t gi = (size_t)y * W + x;
                const int s = sl[gi];
                GV[o] = gn[gi] * (s >= 4 ? inv_q : inv_h);
                SL[o] = s;
            } else {
                GV[o] = 0.f;
                SL[o] = 0;
            }
        }
    }
    __syncthreads();

    // Phase A: per column, VL+VF, VR+VF and VF on rows [qy0, qy1).
    // Blocks of r rows anchored at multiples of r (qy0 is one).
    {
        const int nblk = (qy1 - qy0 + r - 1) / r;
        for (int b = ty; b < nblk; b += 4) {
            const int y0 = qy0 + b * r, y1 = min(y0 + r, qy1);
            for (int x = qx0 - r + tx; x < qx1 + r; x += 64) {
                const float *gc = GV + x;
                const int *sc = SL + x;
                // direct sums at y0: up over [y0-r, y0], down over [y0, y0+r]
                float u1 = 0.f, u3 = 0.f, ud = 0.f, d2 = 0.f, d4 = 0.f, du = 0.f;
                {
                    const int s = sc[(y0 - r) * pitch];
                    const float g = gc[(y0 - r) * pitch];
                    u1 = pick(M_C1, s, g); u3 = pick(M_C3, s, g); ud = pick(M_FD, s, g);
                }
                for (int yy = y0 - r + 1; yy <= y0; ++yy) {
                    const int s = sc[yy * pitch];
                    const float g = gc[yy * pitch];
                    u1 += pick(M_C1, s, g); u3 += pick(M_C3, s, g); ud += pick(M_FD, s, g);
                }
                {
                    const int s = sc[y0 * pitch];
                    const float g = gc[y0 * pitch];
                    d2 = pick(M_C2, s, g); d4 = pick(M_C4, s, g); du = pick(M_FU, s, g);
                }
                for (int yy = y0 + 1; yy <= y0 + r; ++yy) {
                    const int s = sc[yy * pitch];
                    const float g = gc[yy * pitch];
                    d2 += pick(M_C2, s, g); d4 += pick(M_C4, s, g); du += pick(M_FU, s, g);
                }
                for (int y = y0; y < y1; ++y) {
                    if (y > y0) {
                        const int sn = sc[y * pitch], so = sc[(y - r - 1) * pitch];
                        const float gn_ = gc[y * pitch], go = gc[(y - r - 1) * pitch];
                        u1 += pick(M_C1, sn, gn_) - pick(M_C1, so, go);
                        u3 += pick(M_C3, sn, gn_) - pick(M_C3, so, go);
                        ud += pick(M_FD, sn, gn_) - pick(M_FD, so, go);
                        const int sn2 = sc[(y + r) * pitch], so2 = sc[(y - 1) * pitch];
                        const float gn2 = gc[(y + r) * pitch], go2 = gc[(y - 1) * pitch];
                        d2 += pick(M_C2, sn2, gn2) - pick(M_C2, so2, go2);
                        d4 += pick(M_C4, sn2, gn2) - pick(M_C4, so2, go2);
                        du += pick(M_FU, sn2, gn2) - pick(M_FU, so2, go2);
                    }
                    const int s = sc[y * pitch];
                    const float g = gc[y * pitch];
                    const float vf = ud + du;
                    const float vl = u1 + d2 - pick(M_FR, s, g);
                    const float vr = u3 + d4 - pick(M_FL, s, g);
                    const int o = y * pitch + x;
                    HL[o] = vl + vf;
                    HR[o] = vr + vf;
                    VF[o] = vf;
                }
            }
        }
    }
    __syncthreads();

    // Phase B: Gpad = Hl[HL] + Hr[HR] - VF on [qx0, qx1) x [qy0, qy1), into GV.
    {
        const int nblk = (qx1 - qx0 + r - 1) / r;
        const int nrow = qy1 - qy0;
        for (int b = ty; b < nblk; b += 4) {
            const int x0 = qx0 + b * r, x1 = min(x0 + r, qx1);
            for (int rr = tx; rr < nrow; rr += 64) {
                const int y = qy0 + rr;
                const float *hl = HL + y * pitch, *hr = HR + y * pitch, *vf = VF + y * pitch;
                float *gp = GV + y * pitch;
                float sl_ = hl[x0 - r], sr_ = hr[x0];
                for (int xx = x0 - r + 1; xx <= x0; ++xx) sl_ += hl[xx];
                for (int xx = x0 + 1; xx <= x0 + r; ++xx) sr_ += hr[xx];
                gp[x0] = sl_ + sr_ - vf[x0];
                for (int x = x0 + 1; x < x1; ++x) {
                    sl_ += hl[x] - hl[x - r - 1];
                    sr_ += hr[x + r] - hr[x - 1];
                    gp[x] = sl_ + sr_ - vf[x];
                }
            }
        }
    }
    __syncthreads();

    // Phase C: fold the halo onto edge pixels (adjoint of the clamp), store.
    float *g = a.g + plane_off;
    const int xe = min(W, X0 + TW), ye = min(H, Y0 + TH);
    for (int y = Y0 + ty; y < ye; y += 4) {
        const int ya = y == 0 ? -r : y, yb = y == H - 1 ? H - 1 + r : y;
        for (int x = X0 + tx; x < xe; x += 64) {
            const int xa = x == 0 ? -r : x, xb = x == W - 1 ? W - 1 + r : x;
            float acc;
            if (ya == yb && xa == xb) {
                acc = GV[y * pitch + x];
            } else {
                acc = 0.f;
                for (int qy = ya; qy <= yb; ++qy)
                    for (int qx = xa; qx <= xb; ++qx) acc += GV[qy * pitch + qx];
            }
            g[(size_t)y * W + x] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Two-pass adjoint through global memory for radii beyond the LDS-resident
// kernels (r > 16; their tile grown by 2r on every side no longer fits LDS).
// Pass 1, one thread per (F column, block of r q rows): the masked vertical
// sums of adjoint_kernel's phase A for q rows [-r, H + r) and F columns
// [-2r, W + 2r), into three workspace planes (VL+VF, VR+VF, VF).  Pass 2, one
// thread per output pixel: Gpad at every q of its clamp preimage (the
// horizontal sums of phase B, anchored at the same multiples of r), folded
// in phase C's order.  Same FP32 operations and order as adjoint_kernel.
__global__ __launch_bounds__(256) void adjoint_global_vert(const float *gnext, const uint8_t *sel, float *hl,
                                                           float *hr, float *vf, int H, int W, int r) {
    const int FW = W + 4 * r, QH = H + 2 * r;
    const int x = (int)(blockIdx.x * 256 + threadIdx.x) - 2 * r;  // F column
    const int plane = blockIdx.z;
    if (x >= W + 2 * r) return;
    const int nblk = (QH + r - 1) / r;
    for (int b = blockIdx.y; b < nblk; b += gridDim.y) {  // blocks of r q rows
    const int y0 = -r + b * r, y1 = min(y0 + r, H + r);
    const size_t poff = (size_t)plane * H * W;
    const float *gn = gnext + poff;
    const uint8_t *sl = sel + poff;
    const float inv_h = 1.0f / (float)((r + 1) * (2 * r + 1));
    const float inv_q = 1.0f / (float)((r + 1) * (r + 1));
    const bool xin = x >= 0 && x < W;
    auto at = [&](int y, int &s, float &g) {
        if (xin && y >= 0 && y < H) {
            const size_t gi = (size_t)y * W + x;
            s = sl[gi];
            g = gn[gi] * (s >= 4 ? inv_q : inv_h);
        } else {
            s = 0;
            g = 0.f;
        }
    };
    int s;
    float g;
    at(y0 - r, s, g);
    float u1 = pick(M_C1, s, g), u3 = pick(M_C3, s, g), ud = pick(M_FD, s, g);
    for (int yy = y0 - r + 1; yy <= y0; ++yy) {
        at(yy, s, g);
        u1 += pick(M_C1, s, g); u3 += pick(M_C3, s, g); ud += pick(M_FD, s, g);
    }
    at(y0, s, g);
    float d2 = pick(M_C2, s, g), d4 = pick(M_C4, s, g), du = pick(M_FU, s, g);
    for (int yy = y0 + 1; yy <= y0 + r; ++yy) {
        at(yy, s, g);
        d2 += pick(M_C2, s, g); d4 += pick(M_C4, s, g); du += pick(M_FU, s, g);
    }
    const size_t qoff = (size_t)plane * QH * FW;
    for (int y = y0; y < y1; ++y) {
        if (y > y0) {
            int sn, so;
            float gn_, go;
            at(y, sn, gn_);
            at(y - r - 1, so, go);
            u1 += pick(M_C1, sn, gn_) - pick(M_C1, so, go);
            u3 += pick(M_C3, sn, gn_) - pick(M_C3, so, go);
            ud += pick(M_FD, sn, gn_) - pick(M_FD, so, go);
            at(y + r, sn, gn_);
            at(y - 1, so, go);
            d2 += pick(M_C2, sn, gn_) - pick(M_C2, so, go);
            d4 += pick(M_C4, sn, gn_) - pick(M_C4, so, go);
            du += pick(M_FU, sn, gn_) - pick(M_FU, so, go);
        }
        at(y, s, g);
        const float v = ud + du;
        const float vl = u1 + d2 - pick(M_FR, s, g);
        const float vr = u3 + d4 - pick(M_FL, s, g);
        const size_t o = qoff + (size_t)(y + r) * FW + (x + 2 * r);
        hl[o] = vl + v;
        hr[o] = vr + v;
        vf[o] = v;
    }
    }
}

__global__ __launch_bounds__(256) void adjoint_global_horiz(const float *hl, const float *hr, const float *vf,
                                                            float *gout, int H, int W, int r) {
    const int FW = W + 4 * r, QH = H + 2 * r;
    const int x = (int)(blockIdx.x * 256 + threadIdx.x), plane = blockIdx.z;
    if (x >= W) return;
    for (int y = blockIdx.y; y < H; y += gridDim.y) {
    const size_t qoff = (size_t)plane * QH * FW;
    // Gpad at q = (qx, qy): horizontal sums anchored at the multiple of r at
    // or left of qx (a direct sum there, then slides), as phase B
    auto gpad = [&](int qx, int qy) {
        const float *L = hl + qoff + (size_t)(qy + r) * FW + 2 * r;  // + q column
        const float *Rr = hr + qoff + (size_t)(qy + r) * FW + 2 * r;
        const float *V = vf + qoff + (size_t)(qy + r) * FW + 2 * r;
        const int x0 = qx - (((qx % r) + r) % r);
        float sl_ = L[x0 - r], sr_ = Rr[x0];
        for (int xx = x0 - r + 1; xx <= x0; ++xx) sl_ += L[xx];
        for (int xx = x0 + 1; xx <= x0 + r; ++xx) sr_ += Rr[xx];
        for (int xx = x0 + 1; xx <= qx; ++xx) {
            sl_ += L[xx] - L[xx - r - 1];
            sr_ += Rr[xx + r] - Rr[xx - 1];
        }
        return sl_ + sr_ - V[qx];
    };
    const int ya = y == 0 ? -r : y, yb = y == H - 1 ? H - 1 + r : y;
    const int xa = x == 0 ? -r : x, xb = x == W - 1 ? W - 1 + r : x;
    float acc;
    if (ya == yb && xa == xb) {
        acc = gpad(x, y);
    } else {
        acc = 0.f;
        for (int qy = ya; qy <= yb; ++qy)
            for (int qx = xa; qx <= xb; ++qx) acc += gpad(qx, qy);
    }
    gout[(size_t)plane * H * W + (size_t)y * W + x] = acc;
    }
}

size_t adjoint_global_ws_bytes(int planes, int H, int W, int r) {
    return (size_t)3 * planes * (size_t)(H + 2 * r) * (size_t)(W + 4 * r) * sizeof(float);
}

hipError_t launch_adjoint_global(const BwdLaunch &a, float *ws, hipStream_t stream) {
    const size_t plane_q = (size_t)(a.H + 2 * a.r) * (a.W + 4 * a.r);
    float *hl = ws, *hr = ws + plane_q * a.planes, *vf = ws + 2 * plane_q * a.planes;
    const dim3 g1((a.W + 4 * a.r + 255) / 256, std::min((a.H + 2 * a.r + a.r - 1) / a.r, 65535), a.planes);
    hipLaunchKernelGGL(adjoint_global_vert, g1, dim3(256), 0, stream, a.gnext, a.sel, hl, hr, vf, a.H, a.W, a.r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2((a.W + 255) / 256, std::min(a.H, 65535), a.planes);
    hipLaunchKernelGGL(adjoint_global_horiz, g2, dim3(256), 0, stream, hl, hr, vf, a.g, a.H, a.W, a.r);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-geometry adjoint for the common radii.  The LDS region is RW x RH
// pixels (the tile grown by 2R on every side) with a compile-time pitch.  The
// vertical pass gives each lane one region column: for every block of R rows
// its wave owns, the lane loads the block's 3R rows of upstream gradient and
// selection straight from global memory (all loads issued before the first
// wait), forms gv and the masked running sums in registers and writes VL+VF,
// VR+VF and VF to LDS.  The horizontal pass spreads (row, block) pairs over
// all lanes and writes Gpad over VF (each block reads only its own VF
// entries).  Three FP32 arrays, no selection array; the FP32 operations and
// their order are those of adjoint_kernel, so both kernels give the same bits.
template <int R, int RW, int RH, int NT>
__global__ __launch_bounds__(NT) void adjoint_fixed_kernel(BwdLaunch a) {
    extern __shared__ float lds[];
    constexpr int PITCH = RW + 1, ARR = RH * PITCH, NY = NT / RW;
    // blocks of R rows per wave, at most: the q region spans at most RH - 2R rows
    constexpr int MB = ((RH - 2 * R + R - 1) / R + NY - 1) / NY;
    static_assert((RW == 64 || RW == 128) && NT % RW == 0, "whole waves per region row");
    float *const HL = lds;
    float *const HR = lds + ARR;
    float *const VF = lds + 2 * ARR;  // VF, then Gpad
    const int tid = threadIdx.x, lx = tid % RW;
    const int ly = __builtin_amdgcn_readfirstlane(tid / RW);
    const int H = a.H, W = a.W, TW = a.tw, TH = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int t = xcd_remap(blockIdx.x, ntiles * a.planes);
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int X0 = (tile % a.tiles_x) * TW, Y0 = (tile / a.tiles_x) * TH;
    const int ox = X0 - 2 * R, oy = Y0 - 2 * R;  // image coords of LDS (0,0)
    const size_t plane_off = (size_t)plane * H * W;
    const float *gn = a.gnext + plane_off;
    const uint8_t *sl = a.sel + plane_off;

    // q region (tile grown by R beyond every image edge it touches) and the
    // F region it reads (q region grown by R)
    const int qx0 = X0 == 0 ? -R : X0, qx1 = X0 + TW >= W ? W + R : X0 + TW;
    const int qy0 = Y0 == 0 ? -R : Y0, qy1 = Y0 + TH >= H ? H + R : Y0 + TH;
    const int gx0 = qx0 - R, gx1 = qx1 + R;
    const float inv_h = 1.0f / (float)((R + 1) * (2 * R + 1));
    const float inv_q = 1.0f / (float)((R + 1) * (R + 1));
    const int x = ox + lx;

    // Phase A: per column of [qx0 - R, qx1 + R), VL+VF, VR+VF and VF on rows
    // [qy0, qy1) in blocks of R rows anchored at multiples of R; gv is
    // G'(p)/n_m(p) inside the image and 0 outside.
    if (x >= gx0 && x < gx1) {
        const bool xin = x >= 0 && x < W;
        const int xc = min(max(x, 0), W - 1);
        const int nblk = (qy1 - qy0 + R - 1) / R;
        float graw[MB][3 * R];
        uint8_t sraw[MB][3 * R];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = ly + i * NY;
            if (b < nblk) {
                const int y0 = qy0 + b * R;
#pragma unroll
                for (int j = 0; j < 3 * R; ++j) {  // rows y0-R .. y0+2R-1, clamped
                    const size_t gi = (size_t)min(max(y0 - R + j, 0), H - 1) * W + xc;
                    graw[i][j] = gn[gi];
                    sraw[i][j] = sl[gi];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = ly + i * NY;
            if (b >= nblk) break;
            const int y0 = qy0 + b * R;
            const bool full = y0 + R <= qy1;
            float g[3 * R];
            int s[3 * R];
#pragma unroll
            for (int j = 0; j < 3 * R; ++j) {
                const int yy = y0 - R + j;
                const bool in = xin && yy >= 0 && yy < H;
                s[j] = in ? sraw[i][j] : 0;
                g[j] = in ? graw[i][j] * (s[j] >= 4 ? inv_q : inv_h) : 0.f;
            }
            float u1 = pick(M_C1, s[0], g[0]), u3 = pick(M_C3, s[0], g[0]), ud = pick(M_FD, s[0], g[0]);
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                u1 += pick(M_C1, s[j], g[j]);
                u3 += pick(M_C3, s[j], g[j]);
                ud += pick(M_FD, s[j], g[j]);
            }
            float d2 = pick(M_C2, s[R], g[R]), d4 = pick(M_C4, s[R], g[R]), du = pick(M_FU, s[R], g[R]);
#pragma unroll
            for (int j = R + 1; j <= 2 * R; ++j) {
                d2 += pick(M_C2, s[j], g[j]);
                d4 += pick(M_C4, s[j], g[j]);
                du += pick(M_FU, s[j], g[j]);
            }
            auto emit = [&](int tt) {
                const int j = R + tt;
                const float vf = ud + du;
                const float vl = u1 + d2 - pick(M_FR, s[j], g[j]);
                const float vr = u3 + d4 - pick(M_FL, s[j], g[j]);
                const int o = (y0 + tt - oy) * PITCH + lx;
                HL[o] = vl + vf;
                HR[o] = vr + vf;
                VF[o] = vf;
            };
            emit(0);
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (full || y0 + tt < qy1) {
                    const int n = R + tt, od = tt - 1, n2 = 2 * R + tt, od2 = R + tt - 1;
                    u1 += pick(M_C1, s[n], g[n]) - pick(M_C1, s[od], g[od]);
                    u3 += pick(M_C3, s[n], g[n]) - pick(M_C3, s[od], g[od]);
                    ud += pick(M_FD, s[n], g[n]) - pick(M_FD, s[od], g[od]);
                    d2 += pick(M_C2, s[n2], g[n2]) - pick(M_C2, s[od2], g[od2]);
                    d4 += pick(M_C4, s[n2], g[n2]) - pick(M_C4, s[od2], g[od2]);
                    du += pick(M_FU, s[n2], g[n2]) - pick(M_FU, s[od2], g[od2]);
                    emit(tt);
                }
            }
        }
    }
    __syncthreads();

    // Phase B: Gpad = Hl[HL] + Hr[HR] - VF on [qx0, qx1) x [qy0, qy1), over
    // VF; work item = (row, block of R columns), rows fastest.
    {
        const int nrow = qy1 - qy0;
        const int nblk = (qx1 - qx0 + R - 1) / R;
        const int dr = NT % nrow, db = NT / nrow;
        int b = tid / nrow, rr = tid - (tid / nrow) * nrow;
        for (; b < nblk;) {
            const int x0 = qx0 + b * R;
            const int ro = (qy0 + rr - oy) * PITCH - ox;  // + image column
            float hl[2 * R], hr[2 * R];
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) {
                hl[i] = HL[ro + x0 - R + i];                        // x0-R .. x0+R-1
                hr[i] = HR[ro + min(x0 + i, qx1 + R - 1)];          // x0 .. x0+2R-1
            }
            float sl_ = hl[0], sr_ = hr[0];
#pragma unroll
            for (int i = 1; i <= R; ++i) sl_ += hl[i];
#pragma unroll
            for (int i = 1; i <= R; ++i) sr_ += hr[i];
            VF[ro + x0] = sl_ + sr_ - VF[ro + x0];
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (x0 + tt < qx1) {
                    sl_ += hl[R + tt] - hl[tt - 1];
                    sr_ += hr[R + tt] - hr[tt - 1];
                    VF[ro + x0 + tt] = sl_ + sr_ - VF[ro + x0 + tt];
                }
            }
            rr += dr;
            b += db;
            if (rr >= nrow) {
                rr -= nrow;
                ++b;
            }
        }
    }
    __syncthreads();

    // Phase C: fold the halo onto edge pixels (adjoint of the clamp), store.
    const float *GP = VF;
    float *g = a.g + plane_off;
    const int xe = min(W, X0 + TW), ye = min(H, Y0 + TH);
    if (x >= X0 && x < xe) {
        const int xa = x == 0 ? -R : x, xb = x == W - 1 ? W - 1 + R : x;
        for (int y = Y0 + ly; y < ye; y += NY) {
            const int ya = y == 0 ? -R : y, yb = y == H - 1 ? H - 1 + R : y;
            float acc;
            if (ya == yb && xa == xb) {
                acc = GP[(y - oy) * PITCH + lx];
            } else {
                acc = 0.f;
                for (int qy = ya; qy <= yb; ++qy)
                    for (int qx = xa; qx <= xb; ++qx) acc += GP[(qy - oy) * PITCH + (qx - ox)];
            }
            g[(size_t)y * W + x] = acc;
        }
    }
}

// Regions (width x height, 512 threads) of the fixed adjoint kernel; other
// radii take the generic kernel.
struct AdjGeom { int r, rw, rh; };
constexpr AdjGeom kAdjGeoms[] = {{1, 64, 48}, {2, 64, 48}, {3, 64, 48}, {4, 64, 48},
                                 {5, 64, 64}, {8, 64, 64}, {10, 128, 64}, {16, 128, 96}};

static const AdjGeom *adjoint_geom(int r) {
    for (const auto &g : kAdjGeoms)
        if (g.r == r) return &g;
    return nullptr;
}

static size_t adjoint_fixed_lds_bytes(int rw, int rh) { return (size_t)3 * rh * (rw + 1) * sizeof(float); }

bool adjoint_fixed_tile(int r, int *tw, int *th, size_t *lds_bytes) {
    const AdjGeom *g = adjoint_geom(r);
    if (!g) return false;
    *tw = ((g->rw - 4 * r) / r) * r;
    *th = ((g->rh - 4 * r) / r) * r;
    *lds_bytes = adjoint_fixed_lds_bytes(g->rw, g->rh);
    return true;
}

template <int R, int RW, int RH>
static hipError_t launch_adjoint_fixed(const BwdLaunch &a, hipStream_t stream) {
    const size_t lds = adjoint_fixed_lds_bytes(RW, RH);
    const void *fn = (const void *)adjoint_fixed_kernel<R, RW, RH, 512>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    hipLaunchKernelGGL((adjoint_fixed_kernel<R, RW, RH, 512>), dim3(blocks), dim3(512), lds, stream, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row-streaming adjoint.  A workgroup of RW lanes owns a strip of TW output
// columns and a chunk of output rows of one plane (lane = region column
// X0 - 2R + lane) and walks down the chunk's q rows CH = M*R at a time.  Per
// step (q rows [s, s + CH)): the lane's gv and selection rows [s - R, s + CH
// + R) live in a register ring; the vertical pass forms VL+VF, VR+VF and VF
// there, block by block, and writes them to LDS; the horizontal pass (each
// lane's (row, column block) items, the same every step) forms Gpad over VF;
// then each lane folds and stores the output rows these q rows complete.
// The ring's origin advances by CH rows per step, so the step is unrolled
// over the ring period and every ring slot is a compile-time constant; the
// next step's rows are loaded (buffer loads, scalar row offsets) straight
// into the slots of rows the vertical pass no longer needs, and converted to
// gv in place when the step that uses them begins.  VF/Gpad is
// double-buffered by step parity, so a step costs two barriers.  The
// block anchors, the FP32 operations and the fold order are those of the
// tiled adjoint kernels, so the results are bit-identical to theirs.
template <int R, int RW, int M>
__global__ __launch_bounds__(RW) void adjoint_stream_kernel(BwdLaunch a) {
    constexpr int PITCH = RW + 1, CH = M * R;
    constexpr int L = CH + 2 * R;                 // ring rows
    static_assert(M == 1, "one block of R rows per step");
    constexpr int NPH = L / CH;                   // ring period in steps (3)
    extern __shared__ float lds[];
    float *const HL = lds;                   // CH rows
    float *const HR = lds + CH * PITCH;      // CH rows
    float *const VF0 = lds + 2 * CH * PITCH; // 2 x CH rows: VF, then Gpad
    const int lx = threadIdx.x;
    const int H = a.H, W = a.W, TW = a.tw, YC = a.th;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int t = xcd_remap(blockIdx.x, ntiles * a.planes);
    const int plane = t / ntiles, tile = t - plane * ntiles;
    const int chunk = tile / a.tiles_x, strip = tile - chunk * a.tiles_x;
    const int X0 = strip * TW, Y0 = chunk * YC;
    const int ox = X0 - 2 * R;  // image column of LDS column 0
    const int x = ox + lx;

    // q region (the chunk grown by R beyond every image edge it touches) and
    // the F columns it reads
    const int qx0 = X0 == 0 ? -R : X0, qx1 = X0 + TW >= W ? W + R : X0 + TW;
    const int qy0 = Y0 == 0 ? -R : Y0, qy1 = Y0 + YC >= H ? H + R : Y0 + YC;
    const bool vcol = x >= qx0 - R && x < qx1 + R;
    const bool xin = x >= 0 && x < W;
    const int xc = min(max(x, 0), W - 1);
    const int xe = min(W, X0 + TW);
    const bool own = x >= X0 && x < xe;
    const int fxa = x == 0 ? -R : x, fxb = x == W - 1 ? W - 1 + R : x;  // fold columns
    const float inv_h = 1.0f / (float)((R + 1) * (2 * R + 1));
    const float inv_q = 1.0f / (float)((R + 1) * (R + 1));
    const int nsteps = (qy1 - qy0 + CH - 1) / CH;

    // rows this item reads (clamped) and writes, as buffer resources with
    // 32-bit offsets from row0
    const int row0 = max(0, qy0 - R);
    const int row1 = min(H, qy0 + nsteps * CH + R);
    const size_t first = (size_t)plane * H * W + (size_t)row0 * W;
    const uint32_t nrow = (uint32_t)(row1 - row0) * (uint32_t)W;
    const BufRsrc rg = buf_rsrc(a.gnext + first, nrow * 4);
    const BufRsrc rs = buf_rsrc(a.sel + first, nrow);
    const BufRsrc ro_ = buf_rsrc(a.g + first, nrow * 4);
    auto ld_g = [&](int y) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, xc * 4, (clampi(y, 0, H - 1) - row0) * W * 4, 0));
    };
    auto ld_s = [&](int y) {
        return (int)__builtin_amdgcn_raw_buffer_load_b8(rs, xc, (clampi(y, 0, H - 1) - row0) * W, 0);
    };

    // this lane's horizontal items: (row, block of R columns), rows of one
    // block of R rows consecutive, row fastest; CH * nb <= M * (TW + 2R) <=
    // M * RW, so M items per lane cover all
    const int nb = (qx1 - qx0 + R - 1) / R;
    int it_t[M], it_x0[M];
    bool it_ok[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int it = lx + k * RW;
        const int m = it / (R * nb), rem = it - m * (R * nb);
        const int b = rem / R;
        it_ok[k] = it < CH * nb;
        it_t[k] = m * R + (rem - b * R);
        it_x0[k] = qx0 + b * R;
    }

    // ring of gv and selection of rows [s - R, s + CH + R) of this lane's
    // column (selection 0 and gv 0 outside the image); raw loaded values
    // until converted
    float G[L];
    int S_[L];
    auto convert = [&](int slot, int yy) {
        const bool in = xin && yy >= 0 && yy < H;
        const int sr = S_[slot];
        S_[slot] = in ? sr : 0;
        G[slot] = in ? G[slot] * (S_[slot] >= 4 ? inv_q : inv_h) : 0.f;
    };
#pragma unroll
    for (int j = 0; j < L; ++j) {
        G[j] = ld_g(qy0 - R + j);
        S_[j] = ld_s(qy0 - R + j);
    }
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) convert(j, qy0 - R + j);

    float acc = 0.f;  // fold of the output row being accumulated
    auto step = [&](auto ph, int n) {
        constexpr int PH = decltype(ph)::value;
        auto sl = [](int j) { return (j + PH * CH) % L; };  // logical j <-> row s0 - R + j
        const int s0 = qy0 + n * CH;
        float *const VF = VF0 + (n & 1) * CH * PITCH;  // by step parity
        // wave priorities by phase: the VALU-heavy vertical pass fills in (0)
        // behind the horizontal pass between the barriers (2) and the fold
        // and store (1); 32x3x512^2, r = 3: the adjoint 1.8% faster (the
        // forward's order, vertical pass at 1, timed the same as none)
        wave_priority<0>();
#pragma unroll
        for (int j = 0; j < CH; ++j) convert(sl(2 * R + j), s0 + R + j);
        // vertical pass: the operations of adjoint_fixed_kernel's block, for
        // the M blocks of R rows of this step
#pragma unroll
        for (int mb = 0; mb < M; ++mb) {
            const int y0 = s0 + mb * R;
            if (!vcol || y0 >= qy1) continue;  // the row condition is uniform
            auto sv = [&](int j) { return S_[sl(mb * R + j)]; };  // rows [y0 - R, y0 + 2R)
            auto gv = [&](int j) { return G[sl(mb * R + j)]; };
            float u1 = pick(M_C1, sv(0), gv(0)), u3 = pick(M_C3, sv(0), gv(0)), ud = pick(M_FD, sv(0), gv(0));
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                u1 += pick(M_C1, sv(j), gv(j));
                u3 += pick(M_C3, sv(j), gv(j));
                ud += pick(M_FD, sv(j), gv(j));
            }
            float d2 = pick(M_C2, sv(R), gv(R)), d4 = pick(M_C4, sv(R), gv(R)), du = pick(M_FU, sv(R), gv(R));
#pragma unroll
            for (int j = R + 1; j <= 2 * R; ++j) {
                d2 += pick(M_C2, sv(j), gv(j));
                d4 += pick(M_C4, sv(j), gv(j));
                du += pick(M_FU, sv(j), gv(j));
            }
            auto emit = [&](int tt) {
                const int j = R + tt;
                const float vf = ud + du;
                const float vl = u1 + d2 - pick(M_FR, sv(j), gv(j));
                const float vr = u3 + d4 - pick(M_FL, sv(j), gv(j));
                const int o = (mb * R + tt) * PITCH + lx;
                HL[o] = vl + vf;
                HR[o] = vr + vf;
                VF[o] = vf;
            };
            emit(0);
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (y0 + tt < qy1) {  // uniform
                    const int nn = R + tt, od = tt - 1, n2 = 2 * R + tt, od2 = R + tt - 1;
                    u1 += pick(M_C1, sv(nn), gv(nn)) - pick(M_C1, sv(od), gv(od));
                    u3 += pick(M_C3, sv(nn), gv(nn)) - pick(M_C3, sv(od), gv(od));
                    ud += pick(M_FD, sv(nn), gv(nn)) - pick(M_FD, sv(od), gv(od));
                    d2 += pick(M_C2, sv(n2), gv(n2)) - pick(M_C2, sv(od2), gv(od2));
                    d4 += pick(M_C4, sv(n2), gv(n2)) - pick(M_C4, sv(od2), gv(od2));
                    du += pick(M_FU, sv(n2), gv(n2)) - pick(M_FU, sv(od2), gv(od2));
                    emit(tt);
                }
            }
        }
        // the next step's rows [s0 + CH + R, s0 + 2CH + R) into the slots of
        // rows [s0 - R, s0 - R + CH), which the vertical pass no longer needs
        if (n + 1 < nsteps) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                G[sl(j)] = ld_g(s0 + CH + R + j);
                S_[sl(j)] = ld_s(s0 + CH + R + j);
            }
        }
        __syncthreads();
        wave_priority<2>();

        // horizontal pass: Gpad = Hl[HL] + Hr[HR] - VF over VF
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (!it_ok[k] || s0 + it_t[k] >= qy1) continue;
            const int ro = it_t[k] * PITCH - ox;  // + image column
            const int x0 = it_x0[k];
            const float *hlp = HL + ro + x0 - R, *hrp = HR + ro + x0;
            float hl[2 * R], hr[2 * R];
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) {
                hl[i] = hlp[i];
                hr[i] = hrp[i];  // past the F columns only where the slide below is skipped
            }
            float sl_ = hl[0], sr_ = hr[0];
#pragma unroll
            for (int i = 1; i <= R; ++i) sl_ += hl[i];
#pragma unroll
            for (int i = 1; i <= R; ++i) sr_ += hr[i];
            float *vp = VF + ro + x0;
            vp[0] = sl_ + sr_ - vp[0];
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (x0 + tt < qx1) {
                    sl_ += hl[R + tt] - hl[tt - 1];
                    sr_ += hr[R + tt] - hr[tt - 1];
                    vp[tt] = sl_ + sr_ - vp[tt];
                }
            }
        }
        wave_priority<1>();
        __syncthreads();

        // fold and store: q row qy belongs to output row clamp(qy); an output
        // row whose clamp preimage (rows [ya, yb] x columns [fxa, fxb]) is
        // more than the pixel sums it row by row, left to right, from 0
        if (own) {
#pragma unroll
            for (int tt = 0; tt < CH; ++tt) {
                const int qy = s0 + tt;
                if (qy >= qy1) break;  // uniform
                const int yo = min(max(qy, 0), H - 1);
                const int ya = yo == 0 ? -R : yo, yb = yo == H - 1 ? H - 1 + R : yo;
                const float *gp = VF + tt * PITCH - ox;  // + image column
                const int so = (yo - row0) * W * 4;
                if (ya == yb && fxa == fxb) {
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(gp[x]), ro_, x * 4, so, 0);
                } else {
                    if (qy == ya) acc = 0.f;
                    for (int qx = fxa; qx <= fxb; ++qx) acc += gp[qx];
                    if (qy == yb) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc), ro_, x * 4, so, 0);
                }
            }
        }
    };
    for (int n = 0; n < nsteps; n += NPH) {
        static_for<0, NPH>([&](auto ph) {
            if (n + decltype(ph)::value < nsteps) step(ph, n + decltype(ph)::value);
        });
    }
}

// Blocks of R rows per step of the streaming adjoint.  One block is fastest
// at every compiled radius on MI355X (32x3x512x512): longer steps (8-10 rows
// at r <= 5) need more registers and LDS and measured 10-25% slower.
constexpr int adj_step_blocks(int) { return 1; }

// Output rows per workgroup: short chunks give many independent workgroups
// per CU, which hides the step barriers and the loads better than fewer long
// walks (32x3x512^2, 5 adjoint sweeps, MPix*it/s at 64 / 24 rows: r=3
// 257 K / 301 K, r=5 239 K / 263 K, r=10 132 K / 143 K; 8 rows is slower
// again, the 2r warm-up rows of each chunk then dominate).  With the 192-lane
// strips at r=3, 18 / 24 / 30 / 36 rows time within 3% of each other, 24
// first.
constexpr int kAdjStreamRows = 24;

// Strip lanes by radius: 128, except 192 at r=3 and 256 at r=16 (32x3x512^2,
// 24-row chunks, MPix*it/s with 128 / 192 / 256 lanes: r=3 293-299 K / 308 K
// / 270 K, r=5 257 K / 202 K / 228 K, r=16 65 K / 62 K / 75 K).
constexpr int adj_stream_lanes(int r) { return r == 16 ? 256 : r == 3 ? 192 : 128; }

// HL, HR and two VF buffers, CH rows each.
static size_t adjoint_stream_lds_bytes(int r) {
    return (size_t)4 * adj_step_blocks(r) * r * (adj_stream_lanes(r) + 1) * sizeof(float);
}

bool adjoint_stream_tile(int r, int *tw, int *th, size_t *lds_bytes) {
    if (!(r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 10 || r == 16)) return false;
    *tw = ((adj_stream_lanes(r) - 4 * r) / r) * r;
    const int step = adj_step_blocks(r) * r;
    *th = (kAdjStreamRows + step - 1) / step * step;
    *lds_bytes = adjoint_stream_lds_bytes(r);
    return true;
}

template <int R>
static hipError_t launch_adjoint_stream(const BwdLaunch &a, hipStream_t stream) {
    const size_t lds = adjoint_stream_lds_bytes(R);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)adjoint_stream_kernel<R, adj_stream_lanes(R), adj_step_blocks(R)>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    hipLaunchKernelGGL((adjoint_stream_kernel<R, adj_stream_lanes(R), adj_step_blocks(R)>), dim3(blocks),
                       dim3(adj_stream_lanes(R)), lds, stream, a);
    return hipGetLastError();
}

// LDS layout of the adjoint kernel for a TW x TH tile: five arrays covering
// the tile grown by 2r on every side.
void bwd_lds_layout(int tw, int th, int r, int *pitch, int *arr) {
    *pitch = (tw + 4 * r) | 1;
    *arr = (th + 4 * r) * (*pitch);
}

hipError_t launch_adjoint(const BwdLaunch &a, hipStream_t stream) {
    if (a.fixed == 2) {
        switch (a.r) {
            case 1: return launch_adjoint_stream<1>(a, stream);
            case 2: return launch_adjoint_stream<2>(a, stream);
            case 3: return launch_adjoint_stream<3>(a, stream);
            case 4: return launch_adjoint_stream<4>(a, stream);
            case 5: return launch_adjoint_stream<5>(a, stream);
            case 8: return launch_adjoint_stream<8>(a, stream);
            case 10: return launch_adjoint_stream<10>(a, stream);
            case 16: return launch_adjoint_stream<16>(a, stream);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.fixed) {
        switch (a.r) {
            case 1: return launch_adjoint_fixed<1, 64, 48>(a, stream);
            case 2: return launch_adjoint_fixed<2, 64, 48>(a, stream);
            case 3: return launch_adjoint_fixed<3, 64, 48>(a, stream);
            case 4: return launch_adjoint_fixed<4, 64, 48>(a, stream);
            case 5: return launch_adjoint_fixed<5, 64, 64>(a, stream);
            case 8: return launch_adjoint_fixed<8, 64, 64>(a, stream);
            case 10: return launch_adjoint_fixed<10, 128, 64>(a, stream);
            case 16: return launch_adjoint_fixed<16, 128, 96>(a, stream);
            default: return hipErrorInvalidValue;
        }
    }
    const size_t lds = (size_t)5 * a.arr * sizeof(float);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)adjoint_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    hipLaunchKernelGGL(adjoint_kernel, dim3(blocks), dim3(256), lds, stream, a);
    return hipGetLastError();
}

}  // namespace osbf
