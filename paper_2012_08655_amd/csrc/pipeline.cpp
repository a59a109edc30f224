// Host-to-host pipeline: frames held in host memory are uploaded, foveated and
// downloaded, with the upload of one frame, the foveation of the frame before
// it and the download of the one before that running at the same time (the
// paper's per-frame loop moves each frame from pinned host memory to the GPU
// and back, and reports the transfer beside the kernel time: Alg. 1, Sec. 3).
//
// The pipeline owns `depth` device slots (an input and an output buffer each)
// and three streams: uploads, foveation and downloads.  Frame k of the
// pipeline uses slot k mod depth.  Per slot three events order the streams:
//   upload of frame k      waits for the foveation of the slot's previous frame
//                          (which read the slot's input buffer);
//   foveation of frame k   waits for its upload and for the download of the
//                          slot's previous frame (which read the output buffer);
//   download of frame k    waits for its foveation.
// Each ticket also gets an event of its own, recorded after its download, so
// a caller can wait for any frame that is still in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "host.h"

namespace fov {

struct PipeSlot {
    void* din = nullptr;
    void* dout = nullptr;
    hipEvent_t uploaded = nullptr;    // the slot's last upload is complete
    hipEvent_t foveated = nullptr;    // the slot's last foveation is complete (its input is free)
    hipEvent_t downloaded = nullptr;  // the slot's last download is complete (its output is free)
    bool used = false;
};

struct PipelineImpl {
    std::mutex mu;
    int device = 0;
    size_t max_in = 0, max_out = 0;
    hipStream_t up = nullptr, comp = nullptr, down = nullptr;
    std::vector<PipeSlot> slots;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, hipEvent_t> inflight;  // ticket -> completion event (NULL: empty frame)
    std::vector<hipEvent_t> free_events;
};

namespace {

// True when the view's elements fill offsets [0, numel) exactly: one copy of
// numel elements moves the whole frame.
bool dense(const fov_tensor& t) {
    const int64_t ext[4] = {t.n, t.c, t.h, t.w}, st[4] = {t.sn, t.sc, t.sh, t.sw};
    int idx[4] = {0, 1, 2, 3};
    std::sort(idx, idx + 4, [&](int a, int b) { return st[a] < st[b]; });
    int64_t expect = 1;
    for (int k = 0; k < 4; ++k) {
        const int d = idx[k];
        if (ext[d] == 1) continue;
        if (st[d] != expect) return false;
        expect *= ext[d];
    }
    return true;
}

size_t view_bytes(const fov_tensor& t) {
    return (size_t)t.n * t.c * t.h * t.w * dtype_size(t.dtype);
}

void release(PipelineImpl* pl) {
    for (hipStream_t s : {pl->up, pl->comp, pl->down})
        if (s) (void)hipStreamSynchronize(s);
    for (PipeSlot& sl : pl->slots) {
        if (sl.din) (void)hipFree(sl.din);
        if (sl.dout) (void)hipFree(sl.dout);
        for (hipEvent_t e : {sl.uploaded, sl.foveated, sl.downloaded})
            if (e) (void)hipEventDestroy(e);
    }
    for (auto& kv : pl->inflight)
        if (kv.second) (void)hipEventDestroy(kv.second);
    for (hipEvent_t e : pl->free_events) (void)hipEventDestroy(e);
    for (hipStream_t s : {pl->up, pl->comp, pl->down})
        if (s) (void)hipStreamDestroy(s);
    delete pl;
}

// Makes the pipeline's device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace
}  // namespace fov

using namespace fov;

struct fov_pipeline {
    PipelineImpl* impl;
};

extern "C" {

fov_status foveate_pipeline_create(int32_t depth, size_t max_in_bytes, size_t max_out_bytes, fov_pipeline** out) {
    if (!out) return set_error(FOV_EINVAL, "out is NULL");
    *out = nullptr;
    if (depth < 1 || depth > 16) return set_error(FOV_EINVAL, "depth must be in 1..16");
    if (max_in_bytes == 0 || max_out_bytes == 0) return set_error(FOV_EINVAL, "buffer sizes must be > 0");
    PipelineImpl* pl = new PipelineImpl();
    pl->max_in = max_in_bytes;
    pl->max_out = max_out_bytes;
    hipError_t e = hipGetDevice(&pl->device);
    if (e != hipSuccess) {
        release(pl);
        return hip_error(e, "hipGetDevice");
    }
    for (hipStream_t* s : {&pl->up, &pl->comp, &pl->down}) {
        e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            release(pl);
            return hip_error(e, "hipStreamCreate");
        }
    }
    pl->slots.resize(depth);
    for (PipeSlot& sl : pl->slots) {
        e = hipMalloc(&sl.din, max_in_bytes);
        if (e == hipSuccess) e = hipMalloc(&sl.dout, max_out_bytes);
        if (e != hipSuccess) {
            release(pl);
            return set_error(FOV_ENOMEM, std::string("pipeline buffer allocation failed: ") + hipGetErrorString(e));
        }
        for (hipEvent_t* ev : {&sl.uploaded, &sl.foveated, &sl.downloaded}) {
            e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                release(pl);
                return hip_error(e, "hipEventCreate");
            }
        }
    }
    *out = new fov_pipeline{pl};
    return FOV_OK;
}

fov_status foveate_pipeline_submit(fov_pipeline* h, const fov_tensor* host_in, const fov_tensor* host_out,
                                   const fov_params* p, uint64_t* ticket) {
    if (!h || !ticket) return set_error(FOV_EINVAL, "NULL argument");
    PipelineImpl* pl = h->impl;
    bool empty = false;
    fov_status st = prepare(host_in, host_out, p, 1, false, &empty);
    if (st != FOV_OK) return st;
    std::lock_guard<std::mutex> lk(pl->mu);
    if (empty) {
        *ticket = pl->next_ticket++;
        pl->inflight[*ticket] = nullptr;
        return FOV_OK;
    }
    if (host_in->n != 1) return set_error(FOV_EINVAL, "a pipeline frame holds one frame (n == 1)");
    if (!dense(*host_in) || !dense(*host_out))
        return set_error(FOV_ELAYOUT, "pipeline frames must be dense views (their elements fill one block)");
    const size_t bin = view_bytes(*host_in), bout = view_bytes(*host_out);
    if (bin > pl->max_in || bout > pl->max_out)
        return set_error(FOV_EINVAL, "frame larger than the pipeline's buffers");
    DeviceGuard guard(pl->device);
    const uint64_t id = pl->next_ticket;
    PipeSlot& sl = pl->slots[(id - 1) % pl->slots.size()];
    hipError_t e = hipSuccess;
    auto fail = [&](const char* what) { return hip_error(e, what); };
    if (sl.used && (e = hipStreamWaitEvent(pl->up, sl.foveated, 0)) != hipSuccess) return fail("hipStreamWaitEvent(up)");
    if ((e = hipMemcpyAsync(sl.din, host_in->data, bin, hipMemcpyHostToDevice, pl->up)) != hipSuccess)
        return fail("hipMemcpyAsync(upload)");
    if ((e = hipEventRecord(sl.uploaded, pl->up)) != hipSuccess) return fail("hipEventRecord(uploaded)");
    if ((e = hipStreamWaitEvent(pl->comp, sl.uploaded, 0)) != hipSuccess) return fail("hipStreamWaitEvent(comp)");
    if (sl.used && (e = hipStreamWaitEvent(pl->comp, sl.downloaded, 0)) != hipSuccess)
        return fail("hipStreamWaitEvent(comp)");
    // The device views keep the host views' strides: both are dense from offset 0.
    fov_tensor din = *host_in, dout = *host_out;
    din.data = sl.din;
    dout.data = sl.dout;
    std::vector<FrameDesc> frames;
    int dt_in = 0, dt_out = 0;
    if ((st = collect_single(&din, &dout, p, 1, &frames, &dt_in, &dt_out)) != FOV_OK) return st;
    if ((st = run_forward(frames, dt_in, dt_out, pl->comp)) != FOV_OK) return st;
    if ((e = hipEventRecord(sl.foveated, pl->comp)) != hipSuccess) return fail("hipEventRecord(foveated)");
    if ((e = hipStreamWaitEvent(pl->down, sl.foveated, 0)) != hipSuccess) return fail("hipStreamWaitEvent(down)");
    if ((e = hipMemcpyAsync(host_out->data, sl.dout, bout, hipMemcpyDeviceToHost, pl->down)) != hipSuccess)
        return fail("hipMemcpyAsync(download)");
    if ((e = hipEventRecord(sl.downloaded, pl->down)) != hipSuccess) return fail("hipEventRecord(downloaded)");
    hipEvent_t done = nullptr;
    if (!pl->free_events.empty()) {
        done = pl->free_events.back();
        pl->free_events.pop_back();
    } else if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) {
        return fail("hipEventCreate");
    }
    if ((e = hipEventRecord(done, pl->down)) != hipSuccess) {
        pl->free_events.push_back(done);
        return fail("hipEventRecord(ticket)");
    }
    sl.used = true;
    pl->inflight[id] = done;
    pl->next_ticket = id + 1;
    *ticket = id;
    return FOV_OK;
}

fov_status foveate_pipeline_query(fov_pipeline* h, uint64_t ticket, int32_t* done) {
    if (!h || !done) return set_error(FOV_EINVAL, "NULL argument");
    PipelineImpl* pl = h->impl;
    std::lock_guard<std::mutex> lk(pl->mu);
    auto it = pl->inflight.find(ticket);
    if (it == pl->inflight.end()) return set_error(FOV_ENOTICKET, "unknown or retired ticket");
    if (!it->second) {
        *done = 1;
        return FOV_OK;
    }
    const hipError_t e = hipEventQuery(it->second);
    if (e == hipErrorNotReady) {
        *done = 0;
        return FOV_OK;
    }
    if (e != hipSuccess) return hip_error(e, "hipEventQuery");
    *done = 1;
    return FOV_OK;
}

fov_status foveate_pipeline_wait(fov_pipeline* h, uint64_t ticket) {
    if (!h) return set_error(FOV_EINVAL, "NULL argument");
    PipelineImpl* pl = h->impl;
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(pl->mu);
        auto it = pl->inflight.find(ticket);
        if (it == pl->inflight.end()) return set_error(FOV_ENOTICKET, "unknown or retired ticket");
        ev = it->second;
        pl->inflight.erase(it);
    }
    if (!ev) return FOV_OK;
    const hipError_t e = hipEventSynchronize(ev);
    std::lock_guard<std::mutex> lk(pl->mu);
    pl->free_events.push_back(ev);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(ticket)");
    return FOV_OK;
}

fov_status foveate_pipeline_destroy(fov_pipeline* h) {
    if (!h) return set_error(FOV_EINVAL, "NULL argument");
    {
        DeviceGuard guard(h->impl->device);
        release(h->impl);
    }
    delete h;
    return FOV_OK;
}

}  // extern "C"
