// Launchers of the row-streaming forward kernel (osbf_stream_device.h) for the
// exact filter, with and without selection maps.
#include "osbf_stream_device.h"

namespace osbf {

// P and V staging (CH rows each), the Q ring (CH + r rows), H (CH rows).
size_t stream_lds_bytes(int RW, int r) {
    const int ch = stream_step_rows(r);
    return (size_t)(4 * ch + r) * (RW + 1) * sizeof(float);
}

// The fused two-sweep kernel: P, V and H staging (CH rows each) and one Q
// ring (CH + r rows) per sweep.
size_t stream2_lds_bytes(int RW, int r) {
    const int ch = stream_step_rows(r);
    return (size_t)(5 * ch + 2 * r) * (RW + 1) * sizeof(float);
}

bool stream_fusable(int RW, int r) { return stream2_radius(r) && RW >= 5 * r; }

int stream_step(int r) { return stream_step_rows(r); }

hipError_t launch_forward_stream(int dtype, const FwdLaunch &a, hipStream_t s) {
    const bool sel = a.sel != nullptr;
    switch (dtype) {
    case DT_F32: return sel ? launch_stream_r<DT_F32, true, MODE_EXACT>(a, s) : launch_stream_r<DT_F32, false, MODE_EXACT>(a, s);
    case DT_F16: return sel ? launch_stream_r<DT_F16, true, MODE_EXACT>(a, s) : launch_stream_r<DT_F16, false, MODE_EXACT>(a, s);
    default: return sel ? launch_stream_r<DT_BF16, true, MODE_EXACT>(a, s) : launch_stream_r<DT_BF16, false, MODE_EXACT>(a, s);
    }
}

}  // namespace osbf
