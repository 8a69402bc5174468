// morph_apply_static: morph_apply with its workspace taken from a fixed device
// array of this library instead of a caller buffer, for callers that cannot
// allocate device memory.  The kernels are morph_apply's own.
#include "../../include/morph.h"
#include "morph_internal.h"

#include <map>
#include <mutex>

// The intermediate image of opening, closing, top-hat, black-hat and the composed
// gradient.  One copy per GPU, held until the process ends.  In host code this name
// is a host-side stand-in, not a device address: only the pointer that
// hipGetSymbolAddress returns for the current device is ever passed on.
static __device__ __align__(256) uint8_t scratch[MORPH_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr; // device ordinal -> that device's copy of scratch

// Address of the current device's scratch, looked up once per device.
int scratch_for_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return morph::record_hip_error(e);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return MORPH_OK;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return morph::record_hip_error(e != hipSuccess ? e : hipErrorUnknown);
    g_scratch_ptr[dev] = p;
    *out = p;
    return MORPH_OK;
}

} // namespace

extern "C" int morph_apply_static(int op, int dtype, const void *src, void *dst, int H, int W,
                                  size_t pitch, int wx, int wy, int anchor_x, int anchor_y,
                                  int border, const morph_plan *plan, hipStream_t stream)
{
    // erosion and dilation need no workspace: exactly morph_apply
    if (op == MORPH_OP_ERODE || op == MORPH_OP_DILATE)
        return morph_apply(op, dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, border,
                           plan, nullptr, 0, stream);
    if (op < MORPH_OP_ERODE || op > MORPH_OP_BLACKHAT) return MORPH_EINVAL;
    // an intermediate of H rows of `pitch` bytes that does not fit the array:
    // morph_apply returns MORPH_ENOMEM before enqueueing anything
    void *ws = nullptr;
    int rc = scratch_for_current_device(&ws);
    if (rc != MORPH_OK) return rc;
    return morph_apply(op, dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, border, plan,
                       ws, MORPH_STATIC_SCRATCH_BYTES, stream);
}
