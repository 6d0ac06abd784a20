// Allocation-free backprojection, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  It is ctmi_backproject without the workspace argument:
// the interpolated adjoint's brick shells go to a file-scope device array
// instead, one copy per GPU that loads the library, held until the process
// ends.  Every call on a GPU shares that GPU's copy, so calls that overlap
// on one GPU race; each call overwrites the shells it reads (every brick
// writes all of its shell before the neighbours add it), so nothing needs
// clearing between calls.
#include "ctmi_internal.h"

#include <mutex>

namespace ctmi {

namespace {

// 160 MiB: the shells of volumes of up to 75 846 bricks of 16x16x8 voxels
// (a 512^3 volume has 65 536).
constexpr size_t SCRATCH_BYTES = size_t(160) << 20;
__device__ __align__(256) float scratch[SCRATCH_BYTES / sizeof(float)];

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  On the host the array's name is only a
// stand-in for the device symbol, so it is never passed to a kernel: the
// kernels get this address.
hipError_t scratch_address(float** ptr)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static float* addr[MAXDEV] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<float*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace ctmi

extern "C" int ctmi_backproject_noalloc(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0,
                                        int64_t nviews, float beta, void* stream)
{
    int rc;
    if ((rc = ctmi::check_backproject(plan, bp, proj, vol, view0, nviews, beta))) return rc;
    float* ws = nullptr;
    if (bp == CTMI_BP_INTERP) {
        const size_t need = ctmi::interp_adjoint_ws_bytes(*plan);
        if (need > ctmi::SCRATCH_BYTES)
            return ctmi::api_fail(CTMI_EWORKSPACE,
                                  "the volume's brick shells need %zu bytes; the allocation-free backprojection holds "
                                  "%zu (volumes of up to 75846 bricks of 16x16x8 voxels, e.g. 512^3)",
                                  need, ctmi::SCRATCH_BYTES);
        hipError_t e = ctmi::scratch_address(&ws);
        if (e != hipSuccess) return ctmi::api_hip(e, "hipGetSymbolAddress(scratch)");
    }
    return ctmi::run_backproject(plan, bp, proj, vol, view0, nviews, beta, ws, stream);
}
