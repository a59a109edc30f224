// Launch interface of the adjoint (backward) kernel.
#pragma once

#include "common.h"

namespace fov {

size_t adjoint_lds_bytes(int r_cap, int B, int es);
fov_status launch_adjoint_all(const fov_tensor* grad_out, const fov_tensor* grad_in, const fov_params* p,
                              int32_t np, hipStream_t stream, size_t lds_limit);

}  // namespace fov
