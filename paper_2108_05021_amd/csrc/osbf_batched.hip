// Batched forward over many images of different sizes, radii and iteration
// counts, gfx950.
//
// The batch advances in rounds: in every round each unfinished image runs one
// sweep.  A round is one persistent launch: a grid of about one workgroup per
// resident slot on the device walks a work list of (image, item) pairs, an
// item being one row chunk of one strip of one plane (the row-streaming
// kernel's work unit, 128-lane strips), so small and large images share the
// machine without per-image launches.  The host splits each launch's items
// over the 8 XCDs by estimated cost (groups of consecutive items of one image,
// so neighbouring strips meet in one L2, assigned largest first to the least
// loaded XCD); the workgroups of an XCD take its items round-robin.
//
// Every item runs the same code as the single-image streaming kernel; its
// window sums are position-deterministic, so the batch gives the same bits as
// filtering each image alone.  A kernel compiled for radii up to 4 needs far
// fewer registers than one for radii up to 8 (or 16), so a round runs as two
// launches: the items of radius above 4 (listed first) in the larger class,
// then those of radius 1 to 4 in the lean one (the 256-image batch: 401 K
// against 387 K MPix*it/s with the split at radius 2).
#include "osbf_stream_device.h"

namespace osbf {

constexpr int kBatchLanes = 128;

template <int DT, int MAXR>
__device__ __forceinline__ void batched_item(const FwdLaunch &a, int t, float *lds) {
    switch (a.r) {
    case 1: fwd_stream_item<DT, 1, kBatchLanes, stream_step_rows(1), false, MODE_EXACT>(a, t, lds); break;
    case 2: fwd_stream_item<DT, 2, kBatchLanes, stream_step_rows(2), false, MODE_EXACT>(a, t, lds); break;
    case 3:
        if constexpr (MAXR >= 3) fwd_stream_item<DT, 3, kBatchLanes, stream_step_rows(3), false, MODE_EXACT>(a, t, lds);
        break;
    case 4:
        if constexpr (MAXR >= 4) fwd_stream_item<DT, 4, kBatchLanes, stream_step_rows(4), false, MODE_EXACT>(a, t, lds);
        break;
    case 5:
        if constexpr (MAXR >= 5) fwd_stream_item<DT, 5, kBatchLanes, stream_step_rows(5), false, MODE_EXACT>(a, t, lds);
        break;
    case 8:
        if constexpr (MAXR >= 8) fwd_stream_item<DT, 8, kBatchLanes, stream_step_rows(8), false, MODE_EXACT>(a, t, lds);
        break;
    case 10:
        if constexpr (MAXR >= 10) fwd_stream_item<DT, 10, kBatchLanes, stream_step_rows(10), false, MODE_EXACT>(a, t, lds);
        break;
    case 16:
        if constexpr (MAXR >= 16) fwd_stream_item<DT, 16, kBatchLanes, stream_step_rows(16), false, MODE_EXACT>(a, t, lds);
        break;
    default: break;  // rejected on the host
    }
}

// descs: this round's per-image launch descriptors; items: (image, item)
// pairs of this round; bins: the offsets of this launch's 8 XCD bins in
// items, and their end (a cost-balanced static partition made on the host).
template <int DT, int MAXR>
__global__ __launch_bounds__(kBatchLanes) __attribute__((amdgpu_waves_per_eu(stream_min_waves(MAXR))))
void batched_round_kernel(const FwdLaunch *descs, const uint2 *items, const int *bins) {
    extern __shared__ float lds[];
    const int nx = gridDim.x >> 3;           // workgroups per XCD (grid is a multiple of 8)
    const int xcd = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int start = bins[xcd], end = bins[xcd + 1];
    for (int it = start + l; it < end; it += nx) {
        const uint2 w = items[it];
        batched_item<DT, MAXR>(descs[w.x], (int)w.y, lds);
        __syncthreads();  // LDS is reused by the next item
    }
}

int batched_lanes() { return kBatchLanes; }

// LDS of a batch whose largest radius class is maxr: every radius up to it
// must fit (the step, and with it the ring, is not monotonic in r).
size_t batched_lds_bytes(int maxr) {
    size_t b = 0;
    for (int r : {1, 2, 3, 4, 5, 8, 10, 16})
        if (r <= maxr) b = std::max(b, stream_lds_bytes(kBatchLanes, r));
    return b;
}

template <int DT, int MAXR>
static auto batched_kernel() {
    return batched_round_kernel<DT, MAXR>;
}

template <int MAXR>
static const void *batched_fn(int dtype) {
    switch (dtype) {
    case DT_F32: return (const void *)batched_kernel<DT_F32, MAXR>();
    case DT_F16: return (const void *)batched_kernel<DT_F16, MAXR>();
    default: return (const void *)batched_kernel<DT_BF16, MAXR>();
    }
}

// Kernel classes by the largest radius they run: 2 and 4 (about 70 VGPRs, 7
// waves per SIMD), 8 (104, 4 waves) and 16.
static const void *batched_function(int dtype, int maxr) {
    return maxr <= 2   ? batched_fn<2>(dtype)
           : maxr <= 4 ? batched_fn<4>(dtype)
           : maxr <= 8 ? batched_fn<8>(dtype)
                       : batched_fn<16>(dtype);
}

// Resident workgroups of the round kernel on the current device.
hipError_t batched_slots(int dtype, int maxr, int *slots) {
    int dev = 0, cus = 0, per_cu = 0;
    const void *fn = batched_function(dtype, maxr);
    const size_t lds = batched_lds_bytes(maxr);
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && lds > 65536)
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchLanes, lds);
    if (e != hipSuccess) return e;
    *slots = std::max(1, cus * per_cu);
    return hipSuccess;
}

hipError_t launch_batched_round(int dtype, int maxr, const FwdLaunch *descs, const uint2 *items,
                                const int *bins, int grid, hipStream_t stream) {
    const void *fn = batched_function(dtype, maxr);
    const size_t lds = batched_lds_bytes(maxr);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    void *args[] = {(void *)&descs, (void *)&items, (void *)&bins};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kBatchLanes), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace osbf
