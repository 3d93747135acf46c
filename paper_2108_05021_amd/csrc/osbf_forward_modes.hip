// Launchers of the fast approximation (Alg. 3) and of the classical box
// filter, gfx950: the forward kernels of osbf_fwd_device.h instantiated with
// another MODE.  Kept apart from osbf_forward.hip so the two compile in
// parallel.
#include "osbf_fwd_device.h"

namespace osbf {

// The fast approximation (Alg. 3) and the classical box filter: the same
// kernels with another MODE and no maps.  The fast mode needs three LDS
// arrays (no H field).
template <int DT, int R, int RW, int RH, int NT, int MODE>
static hipError_t launch_mode_fixed(const FwdLaunch &a, hipStream_t stream) {
    const size_t lds = (size_t)(MODE == MODE_FAST ? 3 : 4) * RH * (RW + 1) * sizeof(float);
    auto kern = fwd_fixed_kernel<DT, R, RW, RH, NT, false, MODE>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(a.tiles_x * a.tiles_y * a.planes), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

template <int DT, int R, int MODE>
static hipError_t launch_mode_geom(const FwdLaunch &a, hipStream_t s) {
    switch (a.geom) {
    case GEOM_64x48: return launch_mode_fixed<DT, R, 64, 48, 512, MODE>(a, s);
    case GEOM_64x32: return launch_mode_fixed<DT, R, 64, 32, 512, MODE>(a, s);
    case GEOM_64x60: return launch_mode_fixed<DT, R, 64, 60, 512, MODE>(a, s);
    case GEOM_128x64: return launch_mode_fixed<DT, R, 128, 64, 1024, MODE>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int DT, int MODE>
static hipError_t launch_mode_r(const FwdLaunch &a, hipStream_t s) {
    if (a.geom == GEOM_GENERIC) {
        const size_t lds = (size_t)4 * a.arr * sizeof(float);
        auto kern = fwd_tile_kernel<DT, 0, false, MODE>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(a.tiles_x * a.tiles_y * a.planes), dim3(256), lds, s, a);
        return hipGetLastError();
    }
    switch (a.r) {
    case 1: return launch_mode_geom<DT, 1, MODE>(a, s);
    case 2: return launch_mode_geom<DT, 2, MODE>(a, s);
    case 3: return launch_mode_geom<DT, 3, MODE>(a, s);
    case 4: return launch_mode_geom<DT, 4, MODE>(a, s);
    case 5: return launch_mode_geom<DT, 5, MODE>(a, s);
    case 8: return launch_mode_geom<DT, 8, MODE>(a, s);
    case 10: return launch_mode_geom<DT, 10, MODE>(a, s);
    case 16: return launch_mode_geom<DT, 16, MODE>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward_mode(int mode, int dtype, const FwdLaunch &a, hipStream_t s) {
    if (stream_geom(a.geom)) return launch_forward_stream_mode(mode, dtype, a, s);
    if (mode == MODE_FAST) {
        switch (dtype) {
        case DT_F32: return launch_mode_r<DT_F32, MODE_FAST>(a, s);
        case DT_F16: return launch_mode_r<DT_F16, MODE_FAST>(a, s);
        default: return launch_mode_r<DT_BF16, MODE_FAST>(a, s);
        }
    }
    switch (dtype) {
    case DT_F32: return launch_mode_r<DT_F32, MODE_BOX>(a, s);
    case DT_F16: return launch_mode_r<DT_F16, MODE_BOX>(a, s);
    default: return launch_mode_r<DT_BF16, MODE_BOX>(a, s);
    }
}

}  // namespace osbf
