// Launch interface of the adjoint (backward) kernels.
#pragma once

#include "common.h"
#include "forward.h"

namespace fov {

// Shape constants of one adjoint launch (frames, plan and frame table travel
// as for the forward, in a FwdLaunch).
struct AdjShape {
    int32_t bmax;     // largest fragment side
    int32_t sw;       // row stride of the horizontal-transpose scratch: bmax + 2 r_cap
    int32_t cmax;     // largest channel count
    int32_t pitch_a;  // LDS row pitch of the horizontal kernel
    int32_t chunk_c;  // channels the horizontal kernel stages at once
    int32_t pad_b;    // zero rows above and below a staged fragment in the vertical kernel
    int32_t pitch_b;  // LDS column pitch of the vertical kernel
    int32_t tasks_v;  // vertical kernel: output tasks per thread (1, 2 or 4)
    int32_t chunk_v;  // vertical kernel: channels staged together
};

// Leading zero taps before each fragment's weights: windows may start up to
// three taps early (to keep 16-byte LDS loads aligned) and read zeros there.
constexpr int kAdjWeightLead = 4;

AdjShape adjoint_shape(int es, int r_cap, int bmax, int cmax);
size_t adjoint_lds_h(const AdjShape& s, int es);
size_t adjoint_lds_v(const AdjShape& s, int es);
// Scratch elements for nfrag fragments.
size_t adjoint_scratch_elems(const AdjShape& s, int nfrag);

// Horizontal-transpose and vertical-gather kernels after the plan kernel has
// run for `a` (weights at plan.weights + kAdjWeightLead elements, stride
// a.wstride).  es = 4 (float) or 8 (double).
fov_status launch_adjoint(const FwdLaunch& a, const AdjShape& s, int es, const PlanBuffers& plan, void* weights_base,
                          void* scratch, hipStream_t stream, size_t lds_limit);

}  // namespace fov
