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
    int32_t strip_rows;  // padded-tile rows staged in LDS at once
    int32_t wstride;     // weights per fragment in the plan workspace (multiple of 16)
    int32_t blk_prefix[kMaxFramesPerLaunch + 1];
    FrameParams fr[kMaxFramesPerLaunch];
};
static_assert(sizeof(FwdLaunch) <= 4000, "kernel arguments must fit the kernarg segment");

// Plan workspace of one launch: radius per fragment and its normalised taps
// w[0..N) (N = 2r+1, tap k-r at index k), zero-padded to wstride.
struct PlanBuffers {
    int32_t* radius;  // [nfrag]
    int32_t* order;   // [nfrag] fragment ids by decreasing radius (dispatch order)
    void* weights;    // [nfrag][wstride] of float (u8/f32 launches) or double (f64)
};

// Bytes of plan workspace for nfrag fragments, and its layout.
size_t plan_bytes(int nfrag, int wstride, int wsize);
PlanBuffers carve_plan(void* ws, int nfrag);

fov_status launch_forward(const FwdLaunch& a, int nblocks, int in_dtype, int out_dtype, size_t lds,
                          const PlanBuffers& plan, hipStream_t stream, size_t lds_limit);
fov_status launch_plan(const FrameParams& fp, int nblk, double* sigma_out, int32_t* r_out, hipStream_t stream);

// LDS bytes a forward workgroup needs for radius r_cap and fragment side B.
size_t forward_lds_bytes(int in_dtype, int r_cap, int B, int strip_rows);

}  // namespace fov
