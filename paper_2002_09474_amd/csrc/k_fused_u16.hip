// The fused batch dispatch (wave and streaming units in one kernel) for uint16_t images.
#include "morph_device.h"

namespace morph {

hipError_t launch_fused_u16(const FusedTables &t, bool aligned, int lds, hipStream_t stream)
{
    typedef void (*FusedFn)(FusedTables);
    const FusedFn fn = aligned ? batch_fused_kernel<uint16_t, true> : batch_fused_kernel<uint16_t, false>;
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(t.b0[kFusedClasses]), dim3(64), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
