// Launchers of the row-streaming forward kernel (osbf_stream_device.h) for the
// exact filter, with and without selection maps.
#include "osbf_stream_device.h"

namespace osbf {

// P, V and H staging (CH blocks of three rows, block stride 3 (RW + 1) + 30)
// and the Q ring (the register ring's rows, of RW + 1).
size_t stream_lds_bytes(int RW, int r) {
    const int ch = stream_step_rows(r);
    return ((size_t)ch * (3 * (RW + 1) + 30) + (size_t)stream_ring_rows(r, ch) * (RW + 1)) * sizeof(float);
}

// The fused two-sweep kernel: staging of both sweeps' P, their shared V and
// H (CH rows each), one Q ring (CH + r rows) per sweep and the two edge
// columns of the second sweep's input ring.
size_t stream2_lds_bytes(int RW, int r) {
    const int ch = stream_step_rows(r);
    return ((size_t)ch * (4 * (RW + 1) + 29) + (size_t)(2 * ch + 2 * r) * (RW + 1) + 2 * (ch + r)) * sizeof(float);
}

bool stream_fusable(int RW, int r) { return stream2_radius(r) && RW >= 5 * r; }

int stream_step(int r) { return stream_row_quantum(r); }

// Whether a work item of `rows` rows (and its halo) of a plane W elements of
// `es` bytes wide stays within the kernels' 32-bit row offsets.
bool stream_width_ok(int W, int es, int r, int rows) {
    const int ch = stream_step_rows(r);
    return (long long)(rows + 4 * r + 2 * ch) * W * es < (1LL << 31);
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
