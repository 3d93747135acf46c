// Launchers of the row-streaming forward kernel (osbf_stream_device.h) for the
// fast approximation (Alg. 3) and the classical box filter; kept apart from
// osbf_stream.hip so the two compile in parallel.
#include "osbf_stream_device.h"

namespace osbf {

hipError_t launch_forward_stream_mode(int mode, int dtype, const FwdLaunch &a, hipStream_t s) {
    if (mode == MODE_FAST) {
        switch (dtype) {
        case DT_F32: return launch_stream_r<DT_F32, false, MODE_FAST>(a, s);
        case DT_F16: return launch_stream_r<DT_F16, false, MODE_FAST>(a, s);
        default: return launch_stream_r<DT_BF16, false, MODE_FAST>(a, s);
        }
    }
    switch (dtype) {
    case DT_F32: return launch_stream_r<DT_F32, false, MODE_BOX>(a, s);
    case DT_F16: return launch_stream_r<DT_F16, false, MODE_BOX>(a, s);
    default: return launch_stream_r<DT_BF16, false, MODE_BOX>(a, s);
    }
}

}  // namespace osbf
