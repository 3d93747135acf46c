// Launchers of the row-streaming forward kernel (osbf_stream_device.h) for the
// exact filter, with and without selection maps.
#include "osbf_stream_device.h"

namespace osbf {

size_t stream_lds_bytes(int RW, int r) {
    const int ch = stream_step_rows(r);
    return (size_t)(2 * ch + 2 * (ch + r)) * (RW + 1) * sizeof(float);
}

int stream_step(int r) { return stream_step_rows(r); }

// Rows per workgroup measured fastest on MI355X (3x2048x2048 FP32, rows from
// 16 to 96) for the 128- and 256-lane strips; rounded up to whole steps.
int stream_default_rows(int r, int RW) {
    int rows;
    if (RW == 128)
        rows = r == 1 ? 32 : r == 2 ? 32 : r == 3 ? 16 : r == 4 ? 24 : r == 5 ? 48 : r == 8 ? 32 : r == 10 ? 32 : 96;
    else
        rows = r == 1 ? 16 : r == 2 ? 32 : r == 3 ? 32 : r == 4 ? 24 : r == 5 ? 24 : r == 8 ? 32 : r == 10 ? 32 : 64;
    const int step = stream_step_rows(r);
    return (rows + step - 1) / step * step;
}

hipError_t launch_forward_stream(int dtype, const FwdLaunch &a, hipStream_t s) {
    const bool sel = a.sel != nullptr;
    switch (dtype) {
    case DT_F32: return sel ? launch_stream_r<DT_F32, true, MODE_EXACT>(a, s) : launch_stream_r<DT_F32, false, MODE_EXACT>(a, s);
    case DT_F16: return sel ? launch_stream_r<DT_F16, true, MODE_EXACT>(a, s) : launch_stream_r<DT_F16, false, MODE_EXACT>(a, s);
    default: return sel ? launch_stream_r<DT_BF16, true, MODE_EXACT>(a, s) : launch_stream_r<DT_BF16, false, MODE_EXACT>(a, s);
    }
}

}  // namespace osbf
