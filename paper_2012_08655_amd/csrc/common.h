// Internal definitions shared by the HIP sources of libfoveate.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/foveate.h"

namespace fov {

// Frames whose parameters travel in one launch's kernel arguments.
constexpr int kMaxFramesPerLaunch = 32;
// Largest fragment side the kernels accept.
constexpr int kMaxBlock = 64;
// Threads per workgroup of the per-fragment kernels (four wave64s).
constexpr int kThreads = 256;

// One frame's parameters as the device sees them.
struct FrameParams {
    double fix_x, fix_y, e0, slope, cap;
    int32_t block, origin_x, origin_y, nbx;
    const float* sigma_map;
};

// Fragment grid of an h x w frame: columns/rows covering it for a grid whose
// fragment (0,0) starts at (origin_x, origin_y), origin in (-B, 0].
__host__ __device__ inline int grid_extent(int len, int origin, int B) {
    // number of fragments covering [0, len): ceil((len - origin) / B)
    return (len - origin + B - 1) / B;
}

// Blur strength of fragment (bx, by) (Sec. 2: a fragment's blur strength
// follows how far its midpoint lies from the fixation point).
// Midpoint in pixel-centre coordinates; sigma(e) = 0 below e0, else
// min(slope*(e - e0), cap).  IEEE double with no contraction so the host and
// the device produce the same bits; sqrt is correctly rounded on both.
__host__ __device__ inline double fragment_sigma_ramp(const FrameParams& f, int bx, int by) {
#pragma clang fp contract(off)
    double half = (double)(f.block - 1) / 2.0;
    double cx = (double)f.origin_x + (double)bx * (double)f.block + half;
    double cy = (double)f.origin_y + (double)by * (double)f.block + half;
    double dx = cx - f.fix_x;
    double dy = cy - f.fix_y;
    double e = sqrt(dx * dx + dy * dy);
    if (e < f.e0) return 0.0;
    double s = f.slope * (e - f.e0);
    if (s > f.cap) s = f.cap;
    return s > 0.0 ? s : 0.0;
}

// A sigma-map entry clipped to [0, cap]; NaN and negatives mean "copy".
__host__ __device__ inline double clip_map_sigma(double m, double cap) {
    if (!(m > 0.0)) return 0.0;
    double s = m < cap ? m : cap;
    return s > 0.0 ? s : 0.0;
}

// Largest radius radius_of reports.  Far beyond what a workgroup's on-chip
// memory can stage, so a call that reaches it is refused (FOV_ERANGE) rather
// than sized with an overflowed int.
constexpr int kRadiusLimit = 1 << 20;

// Window radius: taps beyond 3 sigma are dropped (Appendix "Methods").  The
// bound is applied in double, before the conversion to int.
__host__ __device__ inline int radius_of(double sigma) {
    if (!(sigma > 0.0)) return 0;
    const double t = ceil(3.0 * sigma);
    return t < (double)kRadiusLimit ? (int)t : kRadiusLimit;
}

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Strided 4-D view as the kernels see it.
struct View {
    void* data;
    int64_t sn, sc, sh, sw;
};

// Thread-local error reporting.
fov_status set_error(fov_status s, const std::string& msg);
fov_status hip_error(hipError_t e, const char* what);

}  // namespace fov
