// Launch interface of the forward and plan kernels.
#pragma once

#include "common.h"

namespace fov {

// Kernel arguments of one forward launch: up to kMaxFramesPerLaunch frames of
// one (c, h, w) shape, each with its own parameters.  Fragments of all frames
// are numbered consecutively; blk_prefix[f] is the first fragment of frame f.
struct FwdLaunch {
    View in, out;
    int32_t c, h, w;
    int32_t nframes;     // frames in this launch
    int32_t frame_base;  // index (along n) of the first frame of this launch
    int32_t r_cap;       // largest radius the LDS allocation was sized for
    int32_t strip_rows;  // tile rows staged in LDS at once
    int32_t pad_;
    int32_t blk_prefix[kMaxFramesPerLaunch + 1];
    FrameParams fr[kMaxFramesPerLaunch];
};
static_assert(sizeof(FwdLaunch) <= 4096, "kernel arguments must fit the 4 KiB kernarg segment");

fov_status launch_forward(const FwdLaunch& a, int nblocks, int in_dtype, int out_dtype, size_t lds,
                          hipStream_t stream, size_t lds_limit);
fov_status launch_plan(const FrameParams& fp, int nblk, double* sigma_out, int32_t* r_out, hipStream_t stream);

}  // namespace fov
