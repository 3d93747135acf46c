// One-sided box filter on volumes (Sec. "Higher Dimension Case"), gfx950.
//
// Fourteen windows per voxel: six halves (one axis one-sided, two full) and
// eight octants (one-sided along all three axes).  Each is a z-sum of a
// planar quantity of the slices it spans:
//   octant (sx,sy,sz) = sum over the sz side in z of the planar quadrant (sx,sy)
//   half +-x / +-y    = sum over the full z range of the planar half
//   half +-z          = sum over the z side of the planar (2r+1)^2 box
// A workgroup (512 or 1024 threads, TH = threads / 64 rows) owns a TW x TH
// column of voxels and a chunk of slices, and streams through the slices
// (2.5D blocking): per slice it loads the clamped
// planar region into LDS, forms the planar running-sum fields V, Q, H of the
// planar kernels, and every thread derives the nine planar quantities of its
// (x, y) column (4 quadrants, 4 halves, the box) into a register ring of the
// last 2r+1 slices.  Once the ring spans [z-r, z+r] the thread sums it along
// z, selects among the 14 windows (scaled distances, tie order +x, -x, +y, -y,
// +z, -z, then octants with x fastest and + first) and writes voxel z.
// The vertical planar pass is fused with the slice load: each lane keeps the
// rows its wave's column blocks need in registers (loaded one slice ahead),
// forms V there and writes its P and V rows to LDS.  P and V are
// double-buffered, so a slice costs two barriers; each voxel's store is
// issued one slice late, ahead of the next slice's loads (loads and stores
// share one memory counter, so the wait for those loads then does not wait
// on fresh stores).
#include "osbf_device.h"
#include "osbf_fwd_device.h"
#include "osbf_internal.h"

#include <cstdlib>

namespace osbf {

// Q on columns [xa, xb+R), rows [ya, yb+R) and H on the same columns, rows
// [ya, yb), like fixed_phase_qh, but with (row, block of R columns) work items
// spread over all lanes: the 3D region is only TH + 2R rows tall.  Blocks run
// fastest, so a wave's lanes read and write along rows (stride R within a
// row, an odd pitch between rows): with rows fastest, lanes one row and one
// block apart hit the same bank.
template <int R, int RW, int NT, bool CL>
__device__ __forceinline__ void phase_qh_items(const float *P, const float *V, float *Q, float *Hs,
                                               int tid, int ox, int oy, int W, int xa, int xb,
                                               int ya, int yb) {
    constexpr int PITCH = RW + 1;
    const int xend = xb + R, yend = yb + R;
    const int nr = yend - ya, nb = (xend - xa + R - 1) / R;
    const int lo = CL ? max(0, xa - R) : xa - R;
    const int hi = CL ? min(W, xend) - 1 : xend - 1;
    const int db = NT % nb, dr = NT / nb;
    int row = tid / nb, b = tid - row * nb;
    while (row < nr) {
        const int y = ya + row;
        const bool doH = y < yb;
        const int x0 = xa + b * R;
        const int rb = (y - oy) * PITCH - ox;  // + image column
        float v[2 * R], p[2 * R];
#pragma unroll
        for (int t = 0; t < 2 * R; ++t) {
            const int col = min(max(x0 - R + t, lo), hi);
            v[t] = V[rb + col];
            p[t] = P[rb + col];
        }
        float q = v[0], h = p[0];
#pragma unroll
        for (int t = 1; t <= R; ++t) {
            q += v[t];
            h += p[t];
        }
        Q[rb + x0] = q;
        if (doH) Hs[rb + x0] = h;
#pragma unroll
        for (int t = 1; t < R; ++t) {
            if (x0 + t < xend) {
                q += v[R + t] - v[t - 1];
                h += p[R + t] - p[t - 1];
                Q[rb + x0 + t] = q;
                if (doH) Hs[rb + x0 + t] = h;
            }
        }
        b += db;
        row += dr;
        if (b >= nb) {
            b -= nb;
            ++row;
        }
    }
}

// Planar quantities of one slice at region offset o: the halves +x, -x, +y,
// -y, the (2R+1)^2 box and the quadrants (+,+), (-,+), (+,-), (-,-).
enum : int { Q_R = 0, Q_L, Q_D, Q_U, Q_BOX, Q_SE, Q_SW, Q_NE, Q_NW, NQ };

template <int R, int PITCH>
__device__ __forceinline__ void planar_quantities(const float *P, const float *V, const float *Q,
                                                  const float *Hs, int o, float q[NQ], float &c) {
    constexpr int RD = R * PITCH;
    c = P[o];
    const float nw = Q[o], ne = Q[o + R], sw = Q[o + RD], se = Q[o + RD + R];
    const float hl = Hs[o], hr = Hs[o + R], vu = V[o], vd = V[o + RD];
    q[Q_R] = ne + se - hr;
    q[Q_L] = nw + sw - hl;
    q[Q_D] = sw + se - vd;
    q[Q_U] = nw + ne - vu;
    q[Q_BOX] = box_sum(nw, ne, sw, se, hl, hr, vu, vd, c);
    q[Q_SE] = se;
    q[Q_SW] = sw;
    q[Q_NE] = ne;
    q[Q_NW] = nw;
}

template <int R, int NT, bool SEL>
__global__ __launch_bounds__(NT) void fwd3d_kernel(Fwd3dLaunch a) {
    constexpr int RW = 64, PITCH = RW + 1, NY = NT / RW, TH = NY, RH = TH + 2 * R;
    constexpr int ARR = RH * PITCH, RING = 2 * R + 1;
    // vertical blocks start at multiples of R at or above the tile's first
    // row: at most TH + 2R - 1 rows of them
    constexpr int MB = ((TH + 2 * R - 1 + R - 1) / R + NY - 1) / NY;  // column blocks per wave, at most
    extern __shared__ float lds[];
    float *const Q = lds + 4 * ARR;
    float *const Hs = lds + 5 * ARR;
    const int tid = threadIdx.x, lx = tid % RW;
    const int ly = __builtin_amdgcn_readfirstlane(tid / RW);
    const int D = a.D, H = a.H, W = a.W, TW = a.tw;
    const int per_vol = a.tiles_x * a.tiles_y * a.chunks;
    const int t = xcd_remap(blockIdx.x, per_vol * a.vols);
    const int vol = t / per_vol;
    int rem = t - vol * per_vol;
    const int chunk = rem / (a.tiles_x * a.tiles_y);
    rem -= chunk * (a.tiles_x * a.tiles_y);
    const int tile_y = rem / a.tiles_x, tile_x = rem - tile_y * a.tiles_x;
    const int X0 = tile_x * TW, Y0 = tile_y * TH;
    const int ox = X0 - R, oy = Y0 - R;
    const int xa = X0, xb = min(W, X0 + TW), ya = Y0, yb = min(H, Y0 + TH);
    const bool interior = X0 - R >= 0 && Y0 - R >= 0 && X0 + TW + R <= W && Y0 + TH + R <= H;
    const int z0 = chunk * a.zc, z1 = min(D, z0 + a.zc);
    const int nsl = (z1 - z0) + 2 * R;  // slices z0-R .. z1+R-1
    const size_t slice = (size_t)H * W;
    const float *src = a.src + (size_t)vol * D * slice;
    float *dst = a.dst + (size_t)vol * D * slice;
    uint8_t *sel = SEL ? a.sel + (size_t)vol * D * slice : nullptr;

    // this thread's (x, y) column; its vertical blocks of R rows (V on rows
    // [yv, yb+R), columns [max(0,xa-R), min(W,xb+R))) and their 2R input
    // rows.  The blocks start at yv, the last multiple of R at or before ya, and
    // the row-sum items at xa, a multiple of R (TW is one), so every running
    // sum restarts at the same image coordinates whatever the tile shape,
    // and a voxel's bits do not depend on the workgroup size or the chunking.
    const int x = ox + lx, y = Y0 + ly;
    const bool own = x >= xa && x < xb && y < yb;
    const bool vx = x >= max(0, xa - R) && x < min(W, xb + R);
    const int yend = yb + R;
    const int yv = ya - ya % R;
    const int nblk = (yend - yv + R - 1) / R;
    float raw[MB][2 * R];
    auto load_rows = [&](int zs) {
        const float *sl_ = src + (size_t)min(max(zs, 0), D - 1) * slice;
        if (vx) {
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int b = ly + i * NY;
                if (b < nblk) {
                    const int y0 = yv + b * R;
#pragma unroll
                    for (int tt = 0; tt < 2 * R; ++tt)
                        raw[i][tt] = sl_[(size_t)min(max(y0 - R + tt, 0), H - 1) * W + x];
                }
            }
        }
    };
    // V and the blocks' own P rows from the registers (the FP32 operations of
    // fixed_phase_v)
    auto v_phase = [&](float *P, float *V) {
        if (!vx) return;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = ly + i * NY;
            if (b >= nblk) break;
            const int y0 = yv + b * R;
            const float *p = raw[i];
#pragma unroll
            for (int tt = 0; tt < R; ++tt) {
                const int yy = y0 + tt;
                if (yy < yend && yy < H) P[(yy - oy) * PITCH + lx] = p[R + tt];
            }
            float *vc = V + (y0 - oy) * PITCH + lx;
            float v = p[0];
#pragma unroll
            for (int tt = 1; tt <= R; ++tt) v += p[tt];
            vc[0] = v;
#pragma unroll
            for (int tt = 1; tt < R; ++tt) {
                if (y0 + tt < yend) {
                    v += p[R + tt] - p[tt - 1];
                    vc[tt * PITCH] = v;
                }
            }
        }
    };

    constexpr float w_h = (float)((R + 1) * (R + 1)), w_o = (float)((2 * R + 1) * (2 * R + 1));
    constexpr float N = (float)((R + 1) * (R + 1) * (R + 1)) * w_o;
    const float invN = 1.0f / N;
    float ring[RING][NQ], cring[RING];

    // deferred store of the previous voxel (value, map index, position)
    float out_v = 0.f;
    int out_i = 0;
    size_t out_at = 0;
    bool out_pending = false;

    load_rows(z0 - R);
    for (int base = 0; base < nsl; base += RING) {
        static_for<0, RING>([&](auto S) {
            constexpr int s = decltype(S)::value;
            const int n = base + s;
            if (n >= nsl) return;  // uniform over the workgroup
            float *P = lds + (n & 1) * ARR;
            float *V = lds + (2 + (n & 1)) * ARR;
            // the phases that end in barriers first, as in the planar kernels
            // (256^3, T=10: r = 1, 2, 3 5%, 11%, 14% faster; the 1024-thread
            // workgroups of r = 4 2% slower, so they keep one priority)
            if constexpr (NT <= 512) wave_priority<1>();
            v_phase(P, V);
            if (out_pending) {
                dst[out_at] = out_v;
                if (SEL) sel[out_at] = (uint8_t)out_i;
                out_pending = false;
            }
            if (n + 1 < nsl) load_rows(z0 - R + n + 1);
            __syncthreads();
            if constexpr (NT <= 512) wave_priority<2>();
            if (interior)
                phase_qh_items<R, RW, NT, false>(P, V, Q, Hs, tid, ox, oy, W, xa, xb, ya, yb);
            else
                phase_qh_items<R, RW, NT, true>(P, V, Q, Hs, tid, ox, oy, W, xa, xb, ya, yb);
            if constexpr (NT <= 512) wave_priority<0>();
            __syncthreads();
            if (!own) return;
            planar_quantities<R, PITCH>(P, V, Q, Hs, (y - oy) * PITCH + lx, ring[s], cring[s]);
            if (n < 2 * R) return;
            // voxel z = z0 + n - 2R: slot of slice z - R + j is (s + 1 + j) % RING
            constexpr int C = (s + 1 + R) % RING;
            const float c = cring[C];
            auto zsum = [&](int k, int j0, int j1) {
                float acc = ring[(s + 1 + j0) % RING][k];
#pragma unroll
                for (int j = j0 + 1; j <= j1; ++j) acc += ring[(s + 1 + j) % RING][k];
                return acc;
            };
            float d[14];
            const float nc = -N * c;
            d[0] = fmaf(w_h, zsum(Q_R, 0, 2 * R), nc);
            d[1] = fmaf(w_h, zsum(Q_L, 0, 2 * R), nc);
            d[2] = fmaf(w_h, zsum(Q_D, 0, 2 * R), nc);
            d[3] = fmaf(w_h, zsum(Q_U, 0, 2 * R), nc);
            d[4] = fmaf(w_h, zsum(Q_BOX, R, 2 * R), nc);
            d[5] = fmaf(w_h, zsum(Q_BOX, 0, R), nc);
            d[6] = fmaf(w_o, zsum(Q_SE, R, 2 * R), nc);
            d[7] = fmaf(w_o, zsum(Q_SW, R, 2 * R), nc);
            d[8] = fmaf(w_o, zsum(Q_NE, R, 2 * R), nc);
            d[9] = fmaf(w_o, zsum(Q_NW, R, 2 * R), nc);
            d[10] = fmaf(w_o, zsum(Q_SE, 0, R), nc);
            d[11] = fmaf(w_o, zsum(Q_SW, 0, R), nc);
            d[12] = fmaf(w_o, zsum(Q_NE, 0, R), nc);
            d[13] = fmaf(w_o, zsum(Q_NW, 0, R), nc);
            // balanced tournament, the lower-numbered entrant wins ties
            float e0 = d[0], e1 = d[2], e2 = d[4], e3 = d[6], e4 = d[8], e5 = d[10], e6 = d[12];
            int i0 = 0, i1 = 2, i2 = 4, i3 = 6, i4 = 8, i5 = 10, i6 = 12;
            duel(e0, i0, d[1], 1);
            duel(e1, i1, d[3], 3);
            duel(e2, i2, d[5], 5);
            duel(e3, i3, d[7], 7);
            duel(e4, i4, d[9], 9);
            duel(e5, i5, d[11], 11);
            duel(e6, i6, d[13], 13);
            duel(e0, i0, e1, i1);
            duel(e2, i2, e3, i3);
            duel(e4, i4, e5, i5);
            duel(e0, i0, e2, i2);
            duel(e4, i4, e6, i6);
            duel(e0, i0, e4, i4);
            const int z = z0 + n - 2 * R;
            out_at = (size_t)z * slice + (size_t)y * W + x;
            out_v = fmaf(e0, invN, c);
            out_i = i0;
            out_pending = true;
        });
    }
    if (out_pending) {
        dst[out_at] = out_v;
        if (SEL) sel[out_at] = (uint8_t)out_i;
    }
}


bool fwd3d_radius(int r) { return r >= 1 && r <= 4; }

// 1024 threads (16-row tiles) halve the planar halo rows per output row;
// measured faster only at r = 4 (98 K against 75 K MVox·it/s on 256^3; at
// r = 4 the 512-thread kernel's 139 VGPRs also leave 3 waves per SIMD), and
// slower at r = 1..3 (186 K / 133 K / 113 K against 193 K / 178 K / 127 K).
int fwd3d_threads(int r) {
    if (const char *env = getenv("OSBF_3D_THREADS")) {
        const int n = atoi(env);
        if (n == 512 || n == 1024) return n;
    }
    return r >= 4 ? 1024 : 512;
}

// Tiles are a multiple of r columns wide (the row sums' anchors).
void fwd3d_geometry(int r, int threads, int *tw, int *th) {
    *tw = (64 - 2 * r) / r * r;
    *th = threads / 64;
}

size_t fwd3d_lds_bytes(int r, int threads) { return (size_t)6 * (threads / 64 + 2 * r) * 65 * sizeof(float); }

template <int R, int NT>
static hipError_t launch3d_nt(const Fwd3dLaunch &a, hipStream_t stream) {
    const int blocks = a.tiles_x * a.tiles_y * a.chunks * a.vols;
    const size_t lds = fwd3d_lds_bytes(R, NT);
    if (a.sel)
        hipLaunchKernelGGL((fwd3d_kernel<R, NT, true>), dim3(blocks), dim3(NT), lds, stream, a);
    else
        hipLaunchKernelGGL((fwd3d_kernel<R, NT, false>), dim3(blocks), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

template <int R>
static hipError_t launch3d(const Fwd3dLaunch &a, hipStream_t stream) {
    if (a.threads == 1024) return launch3d_nt<R, 1024>(a, stream);
    if (a.threads == 512) return launch3d_nt<R, 512>(a, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_forward3d(const Fwd3dLaunch &a, hipStream_t stream) {
    switch (a.r) {
        case 1: return launch3d<1>(a, stream);
        case 2: return launch3d<2>(a, stream);
        case 3: return launch3d<3>(a, stream);
        case 4: return launch3d<4>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace osbf
