// Forward foveation without any allocation: the plan workspace (fragment
// radii, order keys, the queue, the normalised taps and the frame table) lives
// in a fixed array in device memory that the code object declares, instead of
// the per-(device, stream) workspace the library grows with hipMalloc.  Same
// plan, order and main kernels as foveate_forward, so outputs are bitwise the
// same.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host.h"

namespace fov {
namespace {

// Largest plan workspace the array holds.  A 3840x2160 frame in 32 px
// fragments at radius 150 (the widest window a workgroup can stage) needs
// about 10 MiB.
constexpr size_t kScratchBytes = (size_t)16 << 20;

// One copy per device, kept until the process ends.  Host code never passes
// this name to a kernel or a copy: it is a host-side stand-in, and only the
// address hipGetSymbolAddress reports for the current device is a device
// address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's array, looked up once per device
// with that device current.
fov_status scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(FOV_EINVAL, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return set_error(FOV_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FOV_OK;
}

}  // namespace
}  // namespace fov

using namespace fov;

extern "C" fov_status foveate_forward_noalloc(const fov_tensor* in, const fov_tensor* out, const fov_params* p,
                                              int32_t np, void* stream) {
    bool empty = false;
    fov_status s = prepare(in, out, p, np, false, &empty);
    if (s != FOV_OK || empty) return s;
    if (in->n > kArgFrames)
        return set_error(FOV_EINVAL, "foveate_forward_noalloc takes at most " + std::to_string(kArgFrames) +
                                         " frames per call (their descriptors travel in the kernel arguments)");
    FrameDesc frames[kArgFrames];
    for (int i = 0; i < in->n; ++i) frames[i] = make_frame_desc(*in, *out, i, p[np == 1 ? 0 : i]);
    ForwardPlan fp;
    if ((s = plan_forward(frames, in->n, in->dtype, out->dtype, nullptr, &fp)) != FOV_OK) return s;
    const size_t need = fp.pbytes + fp.tbytes;
    if (need > kScratchBytes)
        return set_error(FOV_EINVAL, "this call needs " + std::to_string(need) +
                                         " bytes of plan workspace; foveate_forward_noalloc holds " +
                                         std::to_string(kScratchBytes) + " (use foveate_forward)");
    void* ptr = nullptr;
    if ((s = scratch_of_current_device(&ptr)) != FOV_OK) return s;
    // Every buffer of the plan workspace is written in full by the plan and order kernels before
    // it is read (radii, order keys, every queue slot, every tap, the frame table), so nothing
    // left by an earlier call needs clearing.
    return launch_planned(frames, in->n, in->dtype, out->dtype, fp, ptr, nullptr, (hipStream_t)stream, false);
}
