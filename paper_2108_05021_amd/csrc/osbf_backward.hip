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

// LDS layout of the adjoint kernel for a TW x TH tile: five arrays covering
// the tile grown by 2r on every side.
void bwd_lds_layout(int tw, int th, int r, int *pitch, int *arr) {
    *pitch = (tw + 4 * r) | 1;
    *arr = (th + 4 * r) * (*pitch);
}

hipError_t launch_adjoint(const BwdLaunch &a, hipStream_t stream) {
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
