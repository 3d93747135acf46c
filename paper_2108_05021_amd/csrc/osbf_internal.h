// Internal interfaces between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace osbf {

// One launch of the tiled forward kernel: k fused sweeps over every plane.
struct FwdLaunch {
    const void *src;      // [planes][H][W] storage type
    void *dst;            // [planes][H][W] storage type, never aliases src
    uint8_t *sel;         // nullable; map of this launch's first sweep, plane 0
    long long sel_stride; // elements between consecutive sweeps' maps
    int planes, H, W, r, k;
    int tw, th;           // output tile, multiples of r
    int tiles_x, tiles_y;
    int pitch, arr;       // LDS row pitch and per-array size, in floats
    int geom;             // LDS geometry (Geom)
    // Strided src / dst (the streaming kernels only; 0 = contiguous): row and
    // plane strides in elements.  Maps are always contiguous.
    int src_ld = 0, dst_ld = 0;
    long long src_ps = 0, dst_ps = 0;
};

// LDS geometries: fixed regions compiled for the common radii, the generic
// kernel whose region follows the tile (any radius), or the row-streaming
// kernel (one sweep per launch) whose workgroup walks down a strip of the
// given width.
enum Geom : int { GEOM_GENERIC = 0, GEOM_64x48 = 1, GEOM_64x32 = 2, GEOM_64x60 = 3, GEOM_128x64 = 4,
                  GEOM_S128 = 5, GEOM_S256 = 6, GEOM_S192 = 7, NUM_GEOMS = 8 };
extern const int kGeomDims[NUM_GEOMS][2];   // region width, height (0 for generic and streaming)
bool fixed_radius(int r);
inline bool stream_geom(int g) { return g == GEOM_S128 || g == GEOM_S256 || g == GEOM_S192; }

// Output tile for an LDS region of at most RW x RH pixels (false if none).
bool fwd_tile_shape(int RW, int RH, int r, int k, int *tw, int *th);
void fwd_lds_layout(int tw, int th, int r, int k, int *pitch, int *arr);
hipError_t launch_forward(int dtype, const FwdLaunch &a, hipStream_t s);
// Row-streaming kernel (k = 1, or 2 fused sweeps at small r; any mode):
// strips of tw columns, chunks of th
// rows (th = 0: the launch chooses th so that the chunks fill the device's
// resident workgroup slots once).
int stream_step(int r);                       // th is a multiple (whole steps, whole blocks)
bool stream_width_ok(int W, int es, int r, int rows);  // 32-bit row offsets suffice
size_t stream2_lds_bytes(int RW, int r);      // the fused two-sweep kernel (k = 2)
bool stream_fusable(int RW, int r);           // whether that kernel exists for (RW, r)
size_t stream_lds_bytes(int RW, int r);
hipError_t launch_forward_stream(int dtype, const FwdLaunch &a, hipStream_t s);
hipError_t launch_forward_stream_mode(int mode, int dtype, const FwdLaunch &a, hipStream_t s);
// mode 1: fast approximation (Alg. 3); mode 2: classical box filter.
hipError_t launch_forward_mode(int mode, int dtype, const FwdLaunch &a, hipStream_t s);

// One launch of the adjoint kernel: G = A_t^T Gnext for every plane.
struct BwdLaunch {
    const float *gnext;   // [planes][H][W] upstream gradient G^{t+1}
    const uint8_t *sel;   // [planes][H][W] selection map of forward sweep t
    float *g;             // [planes][H][W] G^t, never aliases gnext
    int planes, H, W, r;
    int tw, th, tiles_x, tiles_y;
    int pitch, arr;       // LDS layout of the generic kernel (bwd_lds_layout)
    int fixed;            // 1: fixed-geometry kernel (adjoint_fixed_tile);
                          // 2: row-streaming kernel (tw strip, th rows per workgroup)
};

void bwd_lds_layout(int tw, int th, int r, int *pitch, int *arr);
// Strip width, rows per workgroup and LDS bytes of the row-streaming adjoint
// for radius r (false if r is not compiled for it).
bool adjoint_stream_tile(int r, int *tw, int *th, size_t *lds_bytes);
// Tile and LDS bytes of the fixed-geometry adjoint kernel for radius r
// (false if r is served by the generic kernel).
bool adjoint_fixed_tile(int r, int *tw, int *th, size_t *lds_bytes);

// Batched rounds (row-streaming work items, batched_lanes()-wide strips); maxr
// is the largest radius the launch runs (selects the kernel class, 2, 4, 8
// or 16, and its LDS); bins (device) holds the offsets of the launch's 8 XCD
// bins in the round's item list and their end.  Items of radius up to
// kBatchLeanMaxR run in a launch of their own, in the lean classes.
constexpr int kBatchLeanMaxR = 4;
int batched_lanes();
size_t batched_lds_bytes(int maxr);
hipError_t batched_slots(int dtype, int maxr, int *slots);
hipError_t launch_batched_round(int dtype, int maxr, const FwdLaunch *descs, const uint2 *items,
                                const int *bins, int grid, hipStream_t stream);
hipError_t launch_adjoint(const BwdLaunch &a, hipStream_t s);
// Radii above kAdjointLdsMaxR: the two-pass adjoint through global memory,
// whose workspace (three planes of the grown q region per plane) is `ws`.
constexpr int kAdjointLdsMaxR = 16;
size_t adjoint_global_ws_bytes(int planes, int H, int W, int r);
hipError_t launch_adjoint_global(const BwdLaunch &a, float *ws, hipStream_t s);

// One sweep of the volume filter over every volume: a workgroup per
// (volume, slice chunk, tile); tiles are tw x (threads / 64) voxel columns.
struct Fwd3dLaunch {
    const float *src;     // [vols][D][H][W]
    float *dst;           // [vols][D][H][W], never aliases src
    uint8_t *sel;         // nullable [vols][D][H][W] map of this sweep
    int vols, D, H, W, r;
    int threads;          // workgroup size: 512 or 1024
    int tw, tiles_x, tiles_y;
    int zc, chunks;       // slices per workgroup, chunks per volume
};
bool fwd3d_radius(int r);
// Workgroup size for radius r (OSBF_3D_THREADS=512|1024 overrides) and the
// tile it owns.
int fwd3d_threads(int r);
void fwd3d_geometry(int r, int threads, int *tw, int *th);
size_t fwd3d_lds_bytes(int r, int threads);
hipError_t launch_forward3d(const Fwd3dLaunch &a, hipStream_t s);

// One sweep of the classical box filter over every plane (the timing
// baseline): strips of tw columns, th rows per workgroup chosen at launch.
struct BoxLaunch {
    const void *src;      // [planes][H][W] storage type
    void *dst;            // [planes][H][W], never aliases src
    int planes, H, W, r;
    int tw, th, tiles_x, tiles_y;
};
bool box_radius(int r);                       // radii of the dedicated kernel
void box_geometry(int r, int *tw, int *step); // strip width, rows per step
hipError_t launch_box(int dtype, const BoxLaunch &a, hipStream_t s);

// One sweep of the one-sided Gaussian filter over every plane.
#define OSBF_GAUSS_MAX_R 8
struct GaussLaunch {
    const float *src;     // [planes][H][W]
    float *dst;           // [planes][H][W], never aliases src
    uint8_t *sel;         // nullable [planes][H][W] map of this sweep
    int planes, H, W, r;
    int tw, th, tiles_x, tiles_y;
    int lanes;            // streaming kernel's strip lanes (tw = lanes - 2r, th = 0: rows
                          // chosen at launch); 0 = tiled kernel
    float g[OSBF_GAUSS_MAX_R + 1];  // taps g(0..r), g(0) = 1
    float w_q, w_h, N, invN;        // distance weights: Zf, Zh, Zh^2 Zf, 1/N
};
bool gauss_radius(int r);
void gauss_tile(int r, int *tw, int *th);
// Kernel and tiling for a.r, a.H, a.W, a.planes (false if the grid is too large).
bool gauss_geometry(GaussLaunch &a);
hipError_t launch_gauss(const GaussLaunch &a, hipStream_t s);

}  // namespace osbf
