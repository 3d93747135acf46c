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

// LDS layout of the adjoint kernel for a TW x TH tile: five arrays covering
// the tile grown by 2r on every side.
void bwd_lds_layout(int tw, int th, int r, int *pitch, int *arr) {
    *pitch = (tw + 4 * r) | 1;
    *arr = (th + 4 * r) * (*pitch);
}

hipError_t launch_adjoint(const BwdLaunch &a, hipStream_t stream) {
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
