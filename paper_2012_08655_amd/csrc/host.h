// Host-side helpers shared by the C ABI entry points and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "forward.h"

namespace fov {

struct DeviceInfo {
    bool ready = false;
    size_t lds_limit = 0;  // dynamic LDS one workgroup may use
    int cus = 0;
    char arch[64] = {0};   // gcnArchName, e.g. "gfx950:sramecc+:xnack-"
};
fov_status device_info(const DeviceInfo** out);

// Per-(device, stream) workspace: device buffer for plans and frame tables,
// pinned host buffer for table uploads (see abi.cpp).
struct Workspace {
    std::mutex mu;  // held by a call from lookup (and any growth) until its launches are enqueued
    void* dev = nullptr;
    size_t dev_bytes = 0;
    void* host = nullptr;
    size_t host_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
};
// The workspace of (current device, stream), grown to at least the given
// sizes, returned with its mutex locked in *hold: host threads that share a
// stream take turns, so none enqueues work with pointers into a buffer
// another thread has just replaced.
fov_status workspace(hipStream_t stream, size_t dev_bytes, size_t host_bytes, Workspace** out,
                     std::unique_lock<std::mutex>* hold);

const std::string& last_error();
int env_int(const char* name, int dflt);

size_t dtype_size(int dt);
bool is_empty(const fov_tensor& t);
fov_status check_view(const fov_tensor* t, const char* name, bool is_output);
fov_status check_alias(const fov_tensor& a, const fov_tensor& b);
fov_status check_params(const fov_params& p, int idx);
FrameParams to_frame(const fov_params& p, int h, int w);
int frame_r_max(const FrameParams& f, int h);
int choose_strip_rows();
bool dispatch_persistent();

// Launch configuration of the forward kernel (public form: fov_tuning).
struct LaunchCfg {
    int split_log2 = 0;
    int strip_rows = 64;
    bool persistent = false;
    int merge = -1;  // vertical pairs at the cap as one item: 1 on, 0 off, -1 on unless it lowers occupancy
    int chan_split = -1;  // small radii one item per channel: 1 on, 0 off, -1 on (several channels)
};

// What a forward call launches: largest radius and fragment side, fragments.
struct CallShape {
    int r_cap = 0, bmax = 1, c = 1;
    int64_t nfrag = 0;
};
CallShape call_shape(const FrameDesc* frames, int nf);

// Configuration for a call: the thread's forced one, else the tuning cache's
// entry for the call's class, else the defaults.
LaunchCfg select_cfg(int nframes, int in_dtype, int out_dtype, const CallShape& cs);

// Validation of a forward (or backward) call's views and parameters.
fov_status prepare(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np, bool backward,
                   bool* empty);
// Descriptor of frame n of a validated (in, out) pair.
FrameDesc make_frame_desc(const fov_tensor& in, const fov_tensor& out, int n, const fov_params& p);
// Argument checks of foveate_forward / foveate_forward_batch, producing the
// frame list (empty frames dropped) and the dtype pair.
fov_status collect_single(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                          std::vector<FrameDesc>* frames, int* dt_in, int* dt_out);
fov_status collect_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps, int32_t nframes,
                         std::vector<FrameDesc>* frames, int* dt_in, int* dt_out);
// Plan, order and main kernels for a list of frames on `stream`, with the
// given configuration (NULL: select_cfg).  profile: take the thread's
// profiler events, if any, for the main kernel.
fov_status run_forward(const std::vector<FrameDesc>& frames, int in_dtype, int out_dtype, hipStream_t stream,
                       const LaunchCfg* cfg = nullptr, bool profile = true);

// The launch shape of one forward call (run_forward in two steps, for callers
// that bring their own plan workspace).
struct ForwardPlan {
    FwdLaunch a;                        // counts and sizes; the frame table is placed by launch_planned
    std::vector<int32_t> prefix_table;  // first fragment of each frame (nframes + 1 entries) when
                                        // nframes > kArgFrames; otherwise they are in a.kprefix
    const int32_t* prefix() const { return a.nframes > kArgFrames ? prefix_table.data() : a.kprefix; }
    size_t lds = 0;               // dynamic LDS per workgroup
    size_t pbytes = 0;            // plan workspace bytes (radii, order keys, queue, taps)
    size_t tbytes = 0;            // frame table bytes, placed after the plan workspace
    size_t lds_limit = 0;
    int cus = 0;
    bool persistent = false;
};
fov_status plan_forward(const FrameDesc* frames, int nf, int in_dtype, int out_dtype, const LaunchCfg* cfg,
                        ForwardPlan* fp);
fov_status launch_planned(const FrameDesc* frames, int nf, int in_dtype, int out_dtype, ForwardPlan& fp,
                          void* scratch, Workspace* ws, hipStream_t stream, bool profile);

}  // namespace fov
