// Launch interface of the adjoint (backward) kernel.
#pragma once

#include "common.h"

namespace fov {

// Kernel arguments of one adjoint launch: up to kMaxFramesPerLaunch frames of
// one (c, h, w) shape; tiles of all frames numbered consecutively.
struct AdjLaunch {
    View in, out;  // grad_out (read), grad_in (written)
    int32_t c, h, w;
    int32_t nframes;
    int32_t frame_base;
    int32_t r_cap;
    int32_t blk_prefix[kMaxFramesPerLaunch + 1];
    FrameParams fr[kMaxFramesPerLaunch];
};
static_assert(sizeof(AdjLaunch) <= 4000, "kernel arguments must fit the kernarg segment");

size_t adjoint_lds_bytes(int r_cap, int B, int es);
fov_status launch_adjoint_all(const fov_tensor* grad_out, const fov_tensor* grad_in, const fov_params* p,
                              int32_t np, hipStream_t stream, size_t lds_limit);

}  // namespace fov
