// The fused batch dispatch (wave and streaming units in one kernel) for uint8_t images.
#include "morph_device.h"

namespace morph {

hipError_t launch_fused_u8(const FusedTables &t, bool aligned, int lds, hipStream_t stream)
{
    typedef void (*FusedFn)(FusedTables);
    const FusedFn fn = aligned ? batch_fused_kernel<uint8_t, true> : batch_fused_kernel<uint8_t, false>;
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(t.b0[kFusedClasses]), dim3(64), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
