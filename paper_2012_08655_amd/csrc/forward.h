// Launch interface of the forward kernels.
#pragma once

#include "common.h"

namespace fov {

// One frame of a forward launch: where it lives, its shape and parameters.
struct FrameDesc {
    const void* in;  // first element of this frame's input
    void* out;       // first element of this frame's output
    int64_t isc, ish, isw, osc, osh, osw;  // element strides
    int32_t c, h, w, nby;
    FrameParams p;  // p.nbx filled in
};

// Frames whose descriptors travel inside the kernel arguments; larger
// batches pass a device table instead.
constexpr int kArgFrames = 16;

// Kernel arguments shared by the plan, order and main forward kernels.
// Fragments of all frames are numbered consecutively: frame f owns fragments
// [prefix[f], prefix[f+1]).  Work item i belongs to fragment i >> (2 split_log2).
struct FwdLaunch {
    int32_t nframes, nfrag;
    int32_t nslots;      // queue slots (work items plus empty padding slots)
    int32_t split_log2;  // each fragment is cut into (2^split_log2)^2 work items (output tiles of
                         // ceil(B / 2^split_log2) pixels a side); 0 = one item per fragment
    int32_t r_cap;       // largest radius the LDS allocation was sized for
    int32_t strip_rows;  // padded-tile rows staged in LDS at once
    int32_t wstride;     // weights per fragment in the plan workspace (multiple of 16)
    int32_t from_args;   // 1: fr[]/kprefix[] hold the frames and the plan kernel
                         // copies them to table/prefix; 0: table/prefix were uploaded
    int32_t cs_rmax;     // >= 0: a fragment with r <= cs_rmax becomes one work item per channel,
                         // its channels in consecutive slots of one XCD after the rest of the
                         // queue, so these short, latency-bound items run their channels side by
                         // side and share that XCD's L2; -1: off.  Needs split_log2 = 0, fewer
                         // than 2^26 fragments and cmax <= 16
    int32_t cmax;        // largest channel count of the frames (with cs_rmax >= 0)
    int32_t merge;       // 1: a fragment at an even row whose sigma and the sigma of the fragment
                         // below both equal the cap becomes one work item with it (equal taps, so
                         // the halo rows they share are computed once); split_log2 must be 0
    FrameDesc* table;    // device table of nframes entries (read by the main kernel)
    int32_t* prefix;     // device array of nframes+1 entries
    const int32_t* hdr;  // optional device header {nframes, nfrag, nslots}: when set, the kernels
                         // read the counts there and the fields above are capacities (a launch
                         // sequence that can be captured once and replayed for many batches; the
                         // replayer sets the main kernel's grid to the batch's slot count)
    int32_t kprefix[kArgFrames + 1];
    FrameDesc fr[kArgFrames];
};
static_assert(sizeof(FwdLaunch) <= 4000, "kernel arguments must fit the kernarg segment");

// Device header of a replayable batch (see FwdLaunch::hdr).
struct BatchHeader {
    int32_t nframes, nfrag, nslots, pad;
};

// Plan workspace of one launch.
struct PlanBuffers {
    int32_t* radius;   // [nfrag] radius of each fragment
    int32_t* okey;     // [nfrag] (ring, angle bin) cell of each fragment for the queue order
    int32_t* order;    // [nslots][2] queue: (work item id, radius word) per slot (id -1 = empty
                       // slot), see the order kernel
    void* weights;     // [nfrag][wstride] normalised taps, float (u8/f32) or double (f64)
};

// Queue slots for nitems work items.
int queue_slots(int nitems, int r_cap);
// Queue slots when fragments may be split by channel (cs_rmax >= 0): room for one slot per
// channel of every fragment and ring padding.
int queue_slots_by_channel(int nfrag, int r_cap, int cmax);
// Order entries of a per-channel work item (cs_rmax >= 0): bit 30 set, channel in bits 26-29,
// fragment in bits 0-25.
constexpr int32_t kChanItem = 1 << 30;
constexpr int kChanShift = 26;
constexpr int32_t kChanItemMask = (1 << kChanShift) - 1;
size_t plan_bytes(int nfrag, int nslots, int wstride, int wsize);
PlanBuffers carve_plan(void* ws, int nfrag, int nslots);

// Plan + order + main kernel for one launch.  persist selects the dispatch of
// the main kernel: a persistent grid striding over the queue, or one
// workgroup per fragment handed out by the hardware dispatcher.
// ev_start/ev_stop, when not null, are recorded on `stream` right before and
// right after the main kernel.
fov_status launch_forward(const FwdLaunch& a, int in_dtype, int out_dtype, size_t lds, const PlanBuffers& plan,
                          hipStream_t stream, size_t lds_limit, int cus, bool persist,
                          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// The main forward kernel for a dtype pair and dispatch mode (to find its node
// in a captured graph); NULL for an unsupported pair.
const void* forward_main_kernel(int in_dtype, int out_dtype, bool persist);

// Device plan for foveate_plan(): sigma and radius of every fragment.
fov_status launch_plan(const FrameParams& fp, int nblk, double* sigma_out, int32_t* r_out, hipStream_t stream);

// LDS bytes a forward workgroup needs for radius r_cap and output tiles of
// tile_w x tile_h pixels (the fragment side B divided by the split, rounded
// up; tile_h = 2B when vertical pairs are merged).
size_t forward_lds_bytes(int in_dtype, int r_cap, int tile_w, int tile_h, int strip_rows);

// Padded-tile rows of a tile tile_h pixels tall at radius r (what a strip
// height above it cannot change).
int forward_tile_rows(int r, int tile_h);

// Workgroups of the main kernel (one workgroup per queue slot) that one CU
// holds at once with `lds` bytes of dynamic LDS each.
int forward_occupancy(int in_dtype, int out_dtype, size_t lds);

// Largest strip height the kernel stages at once.
int forward_strip_max();

// Let `kern` use all the dynamic LDS a workgroup may have on the current
// device (done once per device and kernel; safe to call from any thread).
fov_status allow_dyn_lds(const void* kern, size_t lds_limit);

// Workgroups of kThreads threads with `lds` bytes of dynamic LDS each that
// one CU of the current device holds at once; cached per device, kernel and
// size (safe from any thread); 0 if the query fails.
int occupancy_of(const void* kern, size_t lds);

}  // namespace fov
