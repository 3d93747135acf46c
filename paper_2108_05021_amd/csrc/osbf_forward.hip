// Forward launchers of the one-sided box filter (Alg. 2), gfx950.  The
// kernels themselves live in osbf_fwd_device.h (shared with the batched
// kernel).
#include "osbf_fwd_device.h"

namespace osbf {

template <int DT, int R, bool SEL>
[[maybe_unused]] static hipError_t launch_fwd(const FwdLaunch &a, hipStream_t stream) {
    const size_t lds = (size_t)4 * a.arr * sizeof(float);
    auto kern = fwd_tile_kernel<DT, R, SEL>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, stream, a);
    return hipGetLastError();
}

template <int DT, int R, int RW, int RH, int NT, bool SEL>
static hipError_t launch_fixed(const FwdLaunch &a, hipStream_t stream) {
    const size_t lds = (size_t)4 * RH * (RW + 1) * sizeof(float);
    auto kern = fwd_fixed_kernel<DT, R, RW, RH, NT, SEL>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.tiles_x * a.tiles_y * a.planes;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

template <int DT, int R, bool SEL>
static hipError_t launch_fixed_geom(const FwdLaunch &a, hipStream_t s) {
    switch (a.geom) {
    case GEOM_64x48: return launch_fixed<DT, R, 64, 48, 512, SEL>(a, s);
    case GEOM_64x32: return launch_fixed<DT, R, 64, 32, 512, SEL>(a, s);
    case GEOM_64x60: return launch_fixed<DT, R, 64, 60, 512, SEL>(a, s);
    case GEOM_128x64: return launch_fixed<DT, R, 128, 64, 1024, SEL>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// Selection maps are a training-path feature (FP32 only), so reduced-precision
// launches with maps take the generic kernel (it accepts any layout that fits).
template <int DT, bool SEL>
static hipError_t launch_fwd_r(const FwdLaunch &a, hipStream_t s) {
    if constexpr (SEL && DT != DT_F32) {
        return launch_fwd<DT, 0, SEL>(a, s);
    } else {
    if (a.geom == GEOM_GENERIC) return launch_fwd<DT, 0, SEL>(a, s);
    switch (a.r) {
    case 1: return launch_fixed_geom<DT, 1, SEL>(a, s);
    case 2: return launch_fixed_geom<DT, 2, SEL>(a, s);
    case 3: return launch_fixed_geom<DT, 3, SEL>(a, s);
    case 4: return launch_fixed_geom<DT, 4, SEL>(a, s);
    case 5: return launch_fixed_geom<DT, 5, SEL>(a, s);
    case 8: return launch_fixed_geom<DT, 8, SEL>(a, s);
    case 10: return launch_fixed_geom<DT, 10, SEL>(a, s);
    case 16: return launch_fixed_geom<DT, 16, SEL>(a, s);
    default: return hipErrorInvalidValue;
    }
    }
}

const int kGeomDims[NUM_GEOMS][2] = {{0, 0}, {64, 48}, {64, 32}, {64, 60}, {128, 64}, {128, 0}, {256, 0}, {192, 0}};

bool fixed_radius(int r) {
    return r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 10 || r == 16;
}

hipError_t launch_forward(int dtype, const FwdLaunch &a, hipStream_t s) {
    if (stream_geom(a.geom)) return launch_forward_stream(dtype, a, s);
    const bool sel = a.sel != nullptr;
    switch (dtype) {
    case DT_F32: return sel ? launch_fwd_r<DT_F32, true>(a, s) : launch_fwd_r<DT_F32, false>(a, s);
    case DT_F16: return sel ? launch_fwd_r<DT_F16, true>(a, s) : launch_fwd_r<DT_F16, false>(a, s);
    default: return sel ? launch_fwd_r<DT_BF16, true>(a, s) : launch_fwd_r<DT_BF16, false>(a, s);
    }
}

// Tile shape for a region of at most RW x RH LDS pixels: the output tile is
// the largest multiple of r that leaves room for the k*r halo on both sides.
bool fwd_tile_shape(int RW, int RH, int r, int k, int *tw, int *th) {
    const int w = ((RW - 2 * k * r) / r) * r;
    const int h = ((RH - 2 * k * r) / r) * r;
    if (w < r || h < r || w < 4 || h < 4) return false;
    *tw = w;
    *th = h;
    return true;
}

void fwd_lds_layout(int tw, int th, int r, int k, int *pitch, int *arr) {
    const int ext = k * r;
    *pitch = (tw + 2 * ext) | 1;
    *arr = (th + 2 * ext) * (*pitch);
}

}  // namespace osbf
