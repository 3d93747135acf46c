/*
 * osbf.h -- C ABI of the MI355X (gfx950) one-sided box filter.
 *
 * The filter is Alg. 2 of Gong, "One-Sided Box Filter for Edge Preserving
 * Image Smoothing" (arXiv 2108.05021), Sec. III-A: for every pixel take the
 * means of the eight one-sided windows of Eq. 6-13 (four (r+1)x(r+1)
 * quadrants and four (r+1)x(2r+1) halves, all containing the pixel), replace
 * the pixel by the mean closest to its current value, and repeat.
 *
 * Conventions shared by every entry point
 *   - A plane is H rows by W columns, row-major and contiguous; x is the
 *     column (rightwards), y the row (downwards).  Channels and batch images
 *     are independent planes (the paper filters colour channels separately,
 *     Sec. IV), laid out back to back: element (p, y, x) is at p*H*W + y*W + x.
 *   - Windows, with y pointing down: R = [x, x+r] x [y-r, y+r],
 *     L = [x-r, x] x [y-r, y+r], D = [x-r, x+r] x [y, y+r],
 *     U = [x-r, x+r] x [y-r, y], SE = [x, x+r] x [y, y+r],
 *     SW = [x-r, x] x [y, y+r], NE = [x, x+r] x [y-r, y],
 *     NW = [x-r, x] x [y-r, y].  (The paper's N1..N8 are SW, SE, NE, NW,
 *     L, R, D, U.)  osbf_window numbers them in this order, which is also
 *     the tie order: among windows at the same distance the lowest number
 *     wins.
 *   - Distance: the selection minimises |w_i S_i - N c| over the window sums
 *     S_i, with c the pixel's value, N = (r+1)^2 (2r+1), w_i = 2r+1 for
 *     quadrants and r+1 for halves -- N times the |mean_i - c| of Alg. 2.
 *     Arithmetic is FP32 whatever the storage type, so on integer-valued
 *     images with N * max|value| < 2^24 every comparison is exact.
 *   - Boundary: OSBF_BOUNDARY_REPLICATE reads the replicate extension of the
 *     current iterate at every sweep, U(clamp(x), clamp(y)).
 *   - Iteration: exactly T Jacobi sweeps (sweep t+1 reads sweep t only).
 *     T = 0 or r = 0 is an identity copy.
 *   - Device pointers are plain HIP device (or managed) pointers; `stream`
 *     is a hipStream_t (NULL = the null stream).  Every call is asynchronous
 *     and stream-ordered; the library never allocates, frees or retains
 *     caller memory, and keeps no state beyond a read-only table of tuned
 *     launch shapes.
 *   - Arguments are validated on the host before anything is enqueued; on
 *     error nothing is enqueued and the status says why (see
 *     osbf_last_error() for a message).  Inputs must be finite: NaN or Inf
 *     make the selection unspecified (no fault).
 */
#ifndef OSBF_H
#define OSBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OSBF_ABI_VERSION 2
#define OSBF_MAX_RADIUS 32          /* largest supported r */
#define OSBF3D_MAX_RADIUS 4         /* largest r of the volume filter */
#define OSBF_GAUSS_MAX_RADIUS 8     /* largest r of the one-sided Gaussian filter */

typedef enum {
    OSBF_SUCCESS = 0,
    OSBF_ERROR_INVALID_VALUE = 1,   /* null pointer, bad size, out-of-range enum */
    OSBF_ERROR_UNSUPPORTED = 2,     /* valid request the library has no kernel for */
    OSBF_ERROR_WORKSPACE = 3,       /* workspace missing or too small */
    OSBF_ERROR_HIP = 4,             /* a HIP runtime call or launch failed */
    OSBF_ERROR_TIMEOUT = 5          /* a device-side bounded wait expired */
} osbf_status;

typedef enum {
    OSBF_F32 = 0,                   /* float */
    OSBF_F16 = 1,                   /* IEEE half; iterate rounded to nearest even every sweep */
    OSBF_BF16 = 2                   /* bfloat16; iterate rounded to nearest even every sweep */
} osbf_dtype;

typedef enum { OSBF_BOUNDARY_REPLICATE = 0 } osbf_boundary;

typedef enum {
    OSBF_WIN_R = 0, OSBF_WIN_L = 1, OSBF_WIN_D = 2, OSBF_WIN_U = 3,
    OSBF_WIN_SE = 4, OSBF_WIN_SW = 5, OSBF_WIN_NE = 6, OSBF_WIN_NW = 7
} osbf_window;

/* ABI version (OSBF_ABI_VERSION of the built library). */
int32_t osbf_abi_version(void);

/* Static, never-NULL description of a status code. */
const char *osbf_status_string(osbf_status s);

/* Message of the last failing call on this thread ("" if none). */
const char *osbf_last_error(void);

/*
 * Workspace bytes osbf_forward needs for these sizes (Alg. 2 iterates need one
 * extra plane set to ping-pong through).  Returns 0 when no workspace is
 * needed (T <= 1 with src != dst is served without one) -- callers may always
 * pass at least this many bytes.  Returns (size_t)-1 for invalid sizes.
 */
size_t osbf_forward_workspace_size(int32_t planes, int32_t height, int32_t width,
                                   osbf_dtype dtype, int32_t radius, int32_t iterations);

/*
 * osbf_forward -- T sweeps of Alg. 2 on `planes` independent planes.
 *
 *   src, dst   device, [planes][H][W] of `dtype`; may be equal (in place).
 *   sel        nullable device uint8 [T][planes][H][W]: the window index
 *              (osbf_window) each pixel selected at each sweep.
 *   ckpt       nullable device [ceil(T/ck)][planes][H][W] of `dtype`: the
 *              iterates U^0, U^ck, U^2ck, ... (U^0 is a copy of src), for
 *              recomputing selections in osbf_backward.
 *   ck         checkpoint interval (>= 1) when ckpt is non-NULL, else ignored.
 *   ws         device workspace of ws_bytes >= osbf_forward_workspace_size().
 *
 * The output does not depend on whether sel/ckpt are requested.
 */
osbf_status osbf_forward(const void *src, void *dst, int32_t planes, int32_t height,
                         int32_t width, osbf_dtype dtype, int32_t radius,
                         int32_t iterations, osbf_boundary boundary, uint8_t *sel,
                         void *ckpt, int32_t ck, void *ws, size_t ws_bytes, void *stream);

/*
 * osbf_forward_noalloc -- osbf_forward (no maps, no checkpoints) for callers
 * that cannot allocate device memory: code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It runs the same kernels
 * and gives the same bits as osbf_forward.  The ping-pong iterate lives in a
 * library-owned scratch array of OSBF_NOALLOC_SCRATCH_BYTES per device (held
 * from the first call on a device until the process ends); the call itself
 * allocates nothing.  Images whose plane set exceeds that size
 * (planes*H*W*element bytes) return OSBF_ERROR_WORKSPACE before any launch.
 * Every call on one device shares that device's scratch: calls that overlap
 * in time on one device (different streams or threads) race and must be
 * serialised by the caller.
 */
#define OSBF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
osbf_status osbf_forward_noalloc(const void *src, void *dst, int32_t planes, int32_t height,
                                 int32_t width, osbf_dtype dtype, int32_t radius,
                                 int32_t iterations, osbf_boundary boundary, void *stream);


/*
 * osbf_forward_fast -- T sweeps of the fast approximation of Alg. 3
 * (Sec. III-F): only the north-west quadrant mean field is computed per
 * sweep; the four quadrant candidates are its shifts by {0, r}, and each half
 * window is replaced by the average of its two quadrants (eq:app), so pixels
 * on the shared centre row or column count twice.  The candidate closest to
 * the pixel's value is taken, ties in osbf_window order.  Arguments,
 * boundary, workspace (osbf_forward_workspace_size) and in-place rules as
 * for osbf_forward; no selection maps or checkpoints.
 */
osbf_status osbf_forward_fast(const void *src, void *dst, int32_t planes, int32_t height,
                              int32_t width, osbf_dtype dtype, int32_t radius, int32_t iterations,
                              osbf_boundary boundary, void *ws, size_t ws_bytes, void *stream);

/*
 * osbf_box_forward -- T sweeps of the classical box filter, the mean over the
 * full (2r+1) x (2r+1) window (the baseline the paper times its filter
 * against, Sec. III-G, Table I), with the same boundary, layout, workspace
 * and in-place rules as osbf_forward.
 */
osbf_status osbf_box_forward(const void *src, void *dst, int32_t planes, int32_t height,
                             int32_t width, osbf_dtype dtype, int32_t radius, int32_t iterations,
                             osbf_boundary boundary, void *ws, size_t ws_bytes, void *stream);

/*
 * Workspace bytes osbf_backward needs: one FP32 plane set for the gradient
 * ping-pong, plus (checkpoint mode, ck > 0) two FP32 plane sets and
 * min(ck, T) uint8 maps for recomputing one segment, plus for radii above 16
 * three FP32 planes of (H + 2r) x (W + 4r) per plane for the two-pass
 * adjoint.  (size_t)-1 if invalid.
 */
size_t osbf_backward_workspace_size(int32_t planes, int32_t height, int32_t width,
                                    int32_t radius, int32_t iterations, int32_t ck);

/*
 * osbf_backward -- gradient of T sweeps with every selection held at its
 * forward value (the filter is piecewise linear in the image; away from ties
 * this is its exact derivative).  Each sweep's transpose scatters the
 * upstream gradient of a pixel, divided by the size of its selected window,
 * over that window's clamped pixels; it is computed as a gather (no atomics).
 * Every radius osbf_forward accepts (0..OSBF_MAX_RADIUS): r <= 16 in LDS-
 * resident kernels, larger radii in two passes through the workspace.
 *
 *   grad_out   device FP32 [planes][H][W], gradient w.r.t. the output U^T.
 *   grad_in    device FP32 [planes][H][W], gradient w.r.t. the input U^0;
 *              may equal grad_out.
 *   sel        device uint8 [T][planes][H][W] maps from an FP32 osbf_forward,
 *     or
 *   ckpt, ck   the checkpoints [ceil(T/ck)][planes][H][W] and interval of an
 *              FP32 osbf_forward; each segment's maps are recomputed with the
 *              forward's own kernels (bit-identical to the original maps).
 *              Exactly one of sel / ckpt must be non-NULL (unless T or r is 0).
 *   ws         device workspace >= osbf_backward_workspace_size(..., ck or 0).
 */
osbf_status osbf_backward(const float *grad_out, float *grad_in, int32_t planes, int32_t height,
                          int32_t width, int32_t radius, int32_t iterations,
                          osbf_boundary boundary, const uint8_t *sel, const float *ckpt,
                          int32_t ck, void *ws, size_t ws_bytes, void *stream);

/* One image of a batch: `planes` independent H x W planes, its own radius
 * and iteration count.  src and dst are device pointers and must differ.
 * Strides are in elements, each 0 for the contiguous layout: element
 * (p, y, x) of src is at src + p * src_plane_stride + y * src_row_stride + x
 * (likewise dst), so crops and other views of larger planes are read and
 * written in place.  A non-zero row stride must be >= width, a non-zero
 * plane stride >= height * row stride (planes do not overlap); src and dst
 * must not overlap.  A row stride whose rows overflow the kernels' 32-bit
 * offsets is OSBF_ERROR_UNSUPPORTED.  The library's own extra iterate per
 * image (in the workspace) is contiguous. */
typedef struct {
    const void *src;
    void *dst;
    int32_t planes, height, width, radius, iterations;
    int64_t src_plane_stride, src_row_stride;
    int64_t dst_plane_stride, dst_row_stride;
} osbf_image;

/* A prepared batch (caller-owned plain data; see osbf_batched_prepare). */
typedef struct {
    int32_t n, dtype, rounds, grid;
    int64_t max_items;       /* work items per round, upper bound */
    int64_t total_items;     /* work items over all rounds */
    void *ws;                /* the workspace the tables live in */
    size_t descs_off, items_off, counts_off;
    int32_t identity;        /* images with r = 0 or T = 0 (copied) */
    int32_t reserved[7];
} osbf_batch;

/*
 * Workspace bytes for a batch: one extra iterate per image (ping-pong) plus
 * the per-round descriptor and work tables.  (size_t)-1 if invalid.
 */
size_t osbf_batched_workspace_size(const osbf_image *imgs, int32_t n, osbf_dtype dtype);

/*
 * osbf_batched_prepare -- plan a batch of T_j sweeps of Alg. 2 on each image
 * (all images of one dtype, radii 0..OSBF_MAX_RADIUS) and upload its tables
 * into `ws` on `stream`.  `imgs` is host memory, read during the call.
 * Fills `batch`.  Not capturable into a graph (it copies from host memory).
 * The batched kernels are compiled for r in {1,2,3,4,5,8,10,16}; images of
 * another radius (contiguous planes only, else OSBF_ERROR_UNSUPPORTED) and
 * identity images (r = 0 or T = 0) are left to osbf_batched, which runs
 * them through osbf_forward's launches and copies; osbf_batched_launch
 * refuses a batch that holds any (OSBF_ERROR_UNSUPPORTED).
 */
osbf_status osbf_batched_prepare(const osbf_image *imgs, int32_t n, osbf_dtype dtype,
                                 osbf_boundary boundary, void *ws, size_t ws_bytes,
                                 osbf_batch *batch, void *stream);

/*
 * osbf_batched_launch -- run a prepared batch: per round (every unfinished
 * image advances by one sweep) one persistent launch for the images of
 * radius above 4 and one for those of radius 1 to 4 (a kernel compiled for
 * those radii only, with fewer registers).  Only
 * kernel launches and device-to-device copies are enqueued, so the call can
 * be captured into a HIP graph and replayed; each replay recomputes dst from
 * src.  Results equal per-image osbf_forward bit for bit.
 */
osbf_status osbf_batched_launch(const osbf_batch *batch, void *stream);

/* Prepare and launch in one call; also runs the images the batched kernels
 * do not take (see osbf_batched_prepare), each in its own workspace slice. */
osbf_status osbf_batched(const osbf_image *imgs, int32_t n, osbf_dtype dtype,
                         osbf_boundary boundary, void *ws, size_t ws_bytes, void *stream);

/*
 * osbf_forward_plan -- the launch plan osbf_forward uses for these arguments
 * (for profiling and tests; no device work).  Writes the output tile shape
 * (tiled kernels: tile width x height; row-streaming kernels: strip width x
 * rows per workgroup, 0 = chosen at launch), the sweeps fused per launch (1
 * or 2 for the streaming kernels, 2 only for the fused two-sweep kernel at
 * r <= 5; up to 8 for the tiled kernels) and the number of sweep launches
 * (independent of how the planes are split into grids); ck as for
 * osbf_forward (0 = no checkpoints).  Returns OSBF_ERROR_UNSUPPORTED when no
 * plan fits the device's LDS.
 */
osbf_status osbf_forward_plan(int32_t planes, int32_t height, int32_t width, osbf_dtype dtype,
                              int32_t radius, int32_t iterations, int32_t ck,
                              int32_t *tile_w, int32_t *tile_h, int32_t *fused,
                              int32_t *launches);

/*
 * osbf_autotune -- measure the launch plans of osbf_forward for this problem
 * and keep the fastest for the calling thread's device.
 *   src, dst   distinct device buffers of [planes][height][width] elements of
 *              dtype; src is read, dst is overwritten (scratch)
 * Times every fixed LDS geometry and fusion depth that fits, the
 * row-streaming kernel's strip widths with a few row counts per workgroup,
 * and the cost model's generic plan, with HIP events on `stream`: the
 * candidates back to back, eight launches each, best of three rounds.  The
 * plan the measured tables would use is kept unless another is more than
 * 3% faster.  Blocks until done (do not call during stream capture).  The winner is
 * cached per (device, radius, dtype, size class: planes*height*width below
 * 2^17, below 2^20, up to 2^25, or larger) and used by later osbf_forward / osbf_backward /
 * osbf_forward_plan calls of that class (batches keep their own work
 * items); OSBF_PLAN in the environment still takes precedence.
 * Every plan computes the same bits, so tuning changes speed, never
 * results.  Writes the chosen tile and fused sweeps (0 for
 * radius 0 or iterations 0).  The cache is process state guarded by a mutex.
 */
osbf_status osbf_autotune(const void *src, void *dst, int32_t planes, int32_t height, int32_t width,
                          osbf_dtype dtype, int32_t radius, int32_t iterations, void *stream,
                          int32_t *tile_w, int32_t *tile_h, int32_t *fused);

/*
 * osbf_batched_autotune -- measure the rows per work item of batched launches
 * (osbf_batched_prepare) for the radii of this batch and keep the fastest per
 * (device model, dtype, radius).  Candidates 32, 64 and 128 rows, one radius
 * at a time with the others at their current choice, each timed as the best
 * of three replays of the whole batch after a warm-up; a candidate must beat
 * the incumbent (the cached value, else 64 rows) by 3%.  Overwrites the
 * outputs of the batch (scratch).  ws: device workspace of at least
 * osbf_batched_autotune_workspace_size() bytes.  rows_out (nullable,
 * OSBF_MAX_RADIUS + 1 entries) receives the rows chosen per radius (0 for
 * radii not in the batch).  Blocks until done.  Batches prepared later use
 * the tuned rows; results do not change (work items give the same bits
 * whatever their shape).
 */
size_t osbf_batched_autotune_workspace_size(const osbf_image *imgs, int32_t n, osbf_dtype dtype);
osbf_status osbf_batched_autotune(const osbf_image *imgs, int32_t n, osbf_dtype dtype, void *ws,
                                  size_t ws_bytes, void *stream, int32_t *rows_out);

/*
 * Forget every autotuned plan and batch shape (later calls use the measured
 * tables again).  If OSBF_TUNE_CACHE names a file, the file is kept and read
 * again on the next use of the cache.
 *
 * OSBF_TUNE_CACHE (environment): a file the autotune cache is read from on
 * its first use in a process and written back (whole, atomically replaced)
 * after every osbf_autotune / osbf_batched_autotune call.  Entries are keyed
 * by the device's architecture name and CU count, so the file carries over
 * between processes and machines of one GPU model.  Malformed lines are
 * ignored.
 */
void osbf_autotune_clear(void);

/*
 * Volume filter (Sec. "Higher Dimension Case").  The one-sided kernels along
 * x, y and z span 14 windows per voxel, every one containing the voxel:
 *   0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z   halves: one axis [c, c+r] or
 *                                        [c-r, c], the other two [c-r, c+r];
 *                                        (r+1)(2r+1)^2 voxels
 *   6 (+x,+y,+z), 7 (-x,+y,+z), 8 (+x,-y,+z), 9 (-x,-y,+z),
 *  10 (+x,+y,-z), 11 (-x,+y,-z), 12 (+x,-y,-z), 13 (-x,-y,-z)
 *                                        octants, one-sided on all three axes;
 *                                        (r+1)^3 voxels
 * Each sweep replaces every voxel by the mean of the window whose mean is
 * closest to it (first in the order above on ties), reading the replicate
 * extension of the previous iterate (clamp in x, y and z); T Jacobi sweeps.
 * The index order is this library's reading (the paper names the six halves
 * but orders none of the windows); it extends the planar order.
 */

/* Workspace bytes osbf3d_forward needs (0 if none), (size_t)-1 if invalid. */
size_t osbf3d_forward_workspace_size(int32_t volumes, int32_t depth, int32_t height, int32_t width,
                                     int32_t radius, int32_t iterations);

/*
 * osbf3d_forward -- T sweeps of the volume filter on `volumes` FP32 volumes.
 *   src, dst   device, [volumes][depth][height][width] contiguous FP32
 *              (x fastest, then y, then z); src == dst allowed (in place)
 *   radius     0..OSBF3D_MAX_RADIUS (0 or iterations = 0: copy);
 *              larger radii return OSBF_ERROR_UNSUPPORTED
 *   sel        nullable device [iterations][volumes][depth][height][width]
 *              uint8 window indices (0..13) of every sweep
 *   ws         device workspace of osbf3d_forward_workspace_size bytes
 *              (one FP32 volume set; needed when iterations >= 2 or in place)
 * Stream-ordered and asynchronous; arguments are checked before any launch.
 * Arithmetic is FP32 (sums, selection and means); results match an FP64
 * evaluation up to FP32 rounding and near-tie selections.  The workgroup
 * size (512 threads, 1024 at r = 4) sets where the vertical running sums
 * restart, so OSBF_3D_THREADS=512|1024 in the environment (tests, sweeps)
 * can change the last bits at r = 3.
 */
osbf_status osbf3d_forward(const float *src, float *dst, int32_t volumes, int32_t depth,
                           int32_t height, int32_t width, int32_t radius, int32_t iterations,
                           uint8_t *sel, void *ws, size_t ws_bytes, void *stream);

/*
 * One-sided Gaussian filter (Sec. II-B, separable kernels).  The eight
 * windows, their order and the selection rule are those of osbf_forward; a
 * window's weight at offset (a, b) from the pixel is g(a) g(b) with
 * g(u) = exp(-u^2 / (2 sigma^2)), and its mean is normalised by its own
 * weight total: Zh^2 for quadrants, Zh Zf for halves, Zh = sum_{u=0..r} g(u)
 * and Zf = 2 Zh - 1 (both one-sided parts contain the centre tap, as the
 * box windows do).  sigma = +infinity gives the one-sided box filter.
 */

/* Workspace bytes osbf_gaussian_forward needs (0 if none), (size_t)-1 if invalid. */
size_t osbf_gaussian_workspace_size(int32_t planes, int32_t height, int32_t width, int32_t radius,
                                    int32_t iterations);

/*
 * osbf_gaussian_forward -- T sweeps of the one-sided Gaussian filter on FP32
 * planes.
 *   src, dst   device, [planes][height][width] contiguous FP32; may alias
 *   radius     0..OSBF_GAUSS_MAX_RADIUS (0 or iterations = 0: copy); larger
 *              radii return OSBF_ERROR_UNSUPPORTED (the sums are O(r))
 *   sigma      > 0, +infinity allowed; NaN or <= 0 is OSBF_ERROR_INVALID_VALUE
 *   sel        nullable device [iterations][planes][height][width] uint8
 *              window indices (osbf_window) of every sweep
 *   ws         device workspace of osbf_gaussian_workspace_size bytes (one
 *              FP32 plane set; needed when iterations >= 2 or in place)
 * Replicate boundary at every sweep; stream-ordered and asynchronous;
 * arguments are checked before any launch.  FP32 arithmetic.  Two kernels
 * with bit-identical results: row streaming (default) and 64 x 64 tiles;
 * OSBF_GAUSS=tiled or OSBF_GAUSS=stream[,lanes[,rows]] in the environment
 * selects one (tests, sweeps).
 */
osbf_status osbf_gaussian_forward(const float *src, float *dst, int32_t planes, int32_t height,
                                  int32_t width, int32_t radius, float sigma, int32_t iterations,
                                  uint8_t *sel, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* OSBF_H */
