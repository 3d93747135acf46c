// Batched forward over many images of different sizes, radii and iteration
// counts, gfx950.
//
// The batch advances in rounds: in every round each unfinished image runs its
// own number of fused sweeps (its plan's k, or what is left of T).  A round is
// one persistent launch: a grid of about one workgroup per LDS slot on the
// device walks a work list of (image, plane, tile) items, so small and large
// images share the machine without per-image launches.  Items of a round are
// ordered by decreasing cost, and each XCD takes a contiguous slice of the
// list so neighbouring tiles of an image meet in the same L2.
//
// Every item runs the same fixed-geometry tile code as the single-image
// kernels; its window sums are position-deterministic, so the batch gives the
// same bits as filtering each image alone.
#include "osbf_fwd_device.h"

namespace osbf {

template <int DT>
__device__ __forceinline__ void batched_item(const FwdLaunch &a, int tile, int plane, float *lds) {
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    switch (a.r) {
    case 1: fwd_fixed<DT, 1, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 2: fwd_fixed<DT, 2, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 3: fwd_fixed<DT, 3, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 4: fwd_fixed<DT, 4, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 5: fwd_fixed<DT, 5, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 8: fwd_fixed<DT, 8, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 10: fwd_fixed<DT, 10, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    case 16: fwd_fixed<DT, 16, 64, 48, 512, false>(a, tx, ty, plane, lds); break;
    default: break;  // rejected on the host
    }
}

// descs: this round's per-image launch descriptors; items: (image, item)
// pairs of this round, item = plane * tiles + tile; count: number of items.
template <int DT>
__global__ __launch_bounds__(512) void batched_round_kernel(const FwdLaunch *descs, const uint2 *items,
                                                            const int *count) {
    extern __shared__ float lds[];
    const int n = *count;
    const int nx = gridDim.x >> 3;           // workgroups per XCD (grid is a multiple of 8)
    const int xcd = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int chunk = (n + 7) >> 3;
    const int start = xcd * chunk, end = min(n, start + chunk);
    for (int it = start + l; it < end; it += nx) {
        const uint2 w = items[it];
        const FwdLaunch &a = descs[w.x];
        const int ntiles = a.tiles_x * a.tiles_y;
        const int plane = (int)w.y / ntiles, tile = (int)w.y - plane * ntiles;
        batched_item<DT>(a, tile, plane, lds);
        __syncthreads();  // LDS is reused by the next item
    }
}

size_t batched_lds_bytes() { return (size_t)4 * 48 * 65 * sizeof(float); }

hipError_t launch_batched_round(int dtype, const FwdLaunch *descs, const uint2 *items, const int *count,
                                int grid, hipStream_t stream) {
    const size_t lds = batched_lds_bytes();
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL(batched_round_kernel<DT_F32>, dim3(grid), dim3(512), lds, stream, descs, items, count); break;
    case DT_F16: hipLaunchKernelGGL(batched_round_kernel<DT_F16>, dim3(grid), dim3(512), lds, stream, descs, items, count); break;
    default: hipLaunchKernelGGL(batched_round_kernel<DT_BF16>, dim3(grid), dim3(512), lds, stream, descs, items, count); break;
    }
    return hipGetLastError();
}

}  // namespace osbf
