// Serving: a request table, HBM-budget admission and continuous batching of
// single frames over several HIP streams, with optional hipGraph replay of the
// batch step.  See the serving section of include/foveate.h for the contract.
//
// Threads: callers submit and poll under the server mutex; one scheduler
// thread admits queued frames (FIFO) while the bytes of admitted, unfinished
// frames stay within the budget, and launches everything admitted (up to the
// batch limits) as one batched forward on a free stream; a host function
// queued after each batch marks its frames done and frees the stream, which
// wakes the scheduler.  Frames that arrive while batches run are admitted and
// launched on another stream, so batches overlap on the device.  A frame that
// arrives with a stream free and nothing queued is launched by the submitting
// thread itself, which saves the hand-off to the scheduler.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

namespace fov {
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
    fov_tensor in, out;
    fov_params p;
    hipEvent_t ready = nullptr;  // the caller's producer event (NULL: input already complete)
    size_t bytes = 0;
    int nfrag = 0;
    bool done = false;
    fov_timing t{};
};

struct ServerImpl;

struct Slot {
    ServerImpl* owner = nullptr;
    int index = 0;
    hipStream_t stream = nullptr;  // the slot's own stream (graph capture)
    hipStream_t run = nullptr;     // the stream its batches run on: its own, or slot 0's when shared
    bool busy = false;
    std::vector<uint64_t> tickets;
    size_t bytes = 0;
    int status = FOV_OK;
    // graph replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* dev = nullptr;    // plan workspace + staged batch table
    void* host = nullptr;   // pinned copy of the staged batch table
    size_t stage_bytes = 0;
    hipGraphNode_t main_node = nullptr;  // the main kernel's node: its grid is set per batch
    hipKernelNodeParams main_params{};
};

struct FakeItem {
    double deadline;
    Slot* slot;
};

size_t view_bytes(const fov_tensor& t) {
    if (is_empty(t)) return 0;
    return ((size_t)t.n * t.c * t.h * t.w) * dtype_size(t.dtype);
}

}  // namespace
}  // namespace fov

using namespace fov;

struct fov_server {
    ServerImpl* impl;
};

namespace fov {
namespace {

struct ServerImpl {
    fov_server_cfg cfg{};
    int device = 0;
    int r_cap = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> pending;   // queued, not admitted
    std::deque<uint64_t> admitted;  // admitted, not launched
    size_t inflight_bytes = 0;      // admitted and not done
    uint64_t next_ticket = 1;
    uint64_t batches = 0;
    bool closing = false;
    std::vector<Slot> slots;
    std::thread sched;
    // fake device
    std::thread fake;
    std::deque<FakeItem> fake_q;
    std::condition_variable fake_cv;
    bool fake_stop = false;

    bool fake_mode() const { return cfg.test_fake_device_us > 0; }
    int busy_slots() const {
        int n = 0;
        for (const Slot& s : slots) n += s.busy ? 1 : 0;
        return n;
    }
};

// Completion of a batch (host function queued after it, or the fake device).
void on_batch_done(void* arg) {
    Slot* sl = static_cast<Slot*>(arg);
    ServerImpl* s = sl->owner;
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = now_s();
    for (uint64_t id : sl->tickets) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) continue;
        it->second.done = true;
        it->second.t.t_done = t;
        it->second.t.status = sl->status;
    }
    s->inflight_bytes -= sl->bytes;
    sl->bytes = 0;
    sl->tickets.clear();
    sl->busy = false;
    s->cv.notify_all();
}

void fake_device_loop(ServerImpl* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->fake_cv.wait(lk, [&] { return s->fake_stop || !s->fake_q.empty(); });
        if (s->fake_q.empty() && s->fake_stop) return;
        const FakeItem it = s->fake_q.front();
        s->fake_q.pop_front();
        lk.unlock();
        const double wait = it.deadline - now_s();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        on_batch_done(it.slot);
        lk.lock();
    }
}

// Capacity launch of the replayable batch step of one slot.
FwdLaunch capacity_launch(const ServerImpl* s, const Slot& sl, PlanBuffers* plan, bool merge) {
    FwdLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.merge = merge ? 1 : 0;
    a.cs_rmax = -1;  // whole fragments: batch sizes vary per replay
    a.nframes = s->cfg.max_batch_frames;
    a.nfrag = s->cfg.max_fragments;
    a.nslots = queue_slots(a.nfrag, s->r_cap);
    a.r_cap = s->r_cap;
    a.strip_rows = choose_strip_rows();
    a.wstride = round_up(2 * s->r_cap + 1, 16);
    const int wsize = s->cfg.in_dtype == FOV_F64 ? 8 : 4;
    const size_t pbytes = (plan_bytes(a.nfrag, a.nslots, a.wstride, wsize) + 255) / 256 * 256;
    *plan = carve_plan(sl.dev, a.nfrag, a.nslots);
    char* stage = static_cast<char*>(sl.dev) + pbytes;
    a.hdr = reinterpret_cast<const int32_t*>(stage);
    a.table = reinterpret_cast<FrameDesc*>(stage + sizeof(BatchHeader));
    a.prefix = reinterpret_cast<int32_t*>(stage + sizeof(BatchHeader) + (size_t)a.nframes * sizeof(FrameDesc));
    return a;
}

size_t stage_bytes_of(const fov_server_cfg& c) {
    return sizeof(BatchHeader) + (size_t)c.max_batch_frames * sizeof(FrameDesc) + (size_t)(c.max_batch_frames + 1) * 4;
}

fov_status build_graph(ServerImpl* s, Slot& sl) {
    const DeviceInfo* dev = nullptr;
    fov_status st = device_info(&dev);
    if (st != FOV_OK) return st;
    const int wsize = s->cfg.in_dtype == FOV_F64 ? 8 : 4;
    const int nslots = queue_slots(s->cfg.max_fragments, s->r_cap);
    const int wstride = round_up(2 * s->r_cap + 1, 16);
    const size_t pbytes = (plan_bytes(s->cfg.max_fragments, nslots, wstride, wsize) + 255) / 256 * 256;
    sl.stage_bytes = stage_bytes_of(s->cfg);
    hipError_t e = hipMalloc(&sl.dev, pbytes + sl.stage_bytes);
    if (e != hipSuccess) return set_error(FOV_ENOMEM, "server workspace allocation failed");
    e = hipHostMalloc(&sl.host, sl.stage_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return set_error(FOV_ENOMEM, "server staging allocation failed");
    std::memset(sl.host, 0, sl.stage_bytes);
    // capped vertical pairs as one item (as the plain forward does by default) when the taller
    // tiles let as many workgroups share a CU
    const int B = s->cfg.max_block, sr = choose_strip_rows();
    size_t lds = forward_lds_bytes(s->cfg.in_dtype, s->r_cap, B, B, sr);
    if (lds + 64 > dev->lds_limit) return set_error(FOV_ERANGE, "max_sigma needs more LDS than a workgroup may use");
    const size_t lds2 = forward_lds_bytes(s->cfg.in_dtype, s->r_cap, B, 2 * B, sr);
    const bool merge = s->r_cap > 0 && lds2 + 64 <= dev->lds_limit &&
                       forward_occupancy(s->cfg.in_dtype, s->cfg.out_dtype, lds2) >=
                           forward_occupancy(s->cfg.in_dtype, s->cfg.out_dtype, lds);
    if (merge) lds = lds2;
    PlanBuffers plan;
    const FwdLaunch a = capacity_launch(s, sl, &plan, merge);
    e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    e = hipMemcpyAsync(const_cast<int32_t*>(a.hdr), sl.host, sl.stage_bytes, hipMemcpyHostToDevice, sl.stream);
    st = e == hipSuccess ? FOV_OK : hip_error(e, "hipMemcpyAsync(batch table)");
    if (st == FOV_OK)
        st = launch_forward(a, s->cfg.in_dtype, s->cfg.out_dtype, lds, plan, sl.stream, dev->lds_limit, dev->cus, false);
    if (st == FOV_OK) {
        e = hipLaunchHostFunc(sl.stream, on_batch_done, &sl);
        if (e != hipSuccess) st = hip_error(e, "hipLaunchHostFunc");
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(sl.stream, &g);
    if (st != FOV_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e2 != hipSuccess) return hip_error(e2, "hipStreamEndCapture");
    sl.graph = g;
    // The main kernel was captured with one workgroup per slot of the largest
    // batch; each replay sets its grid to the batch's own slot count.
    const void* main_fn = forward_main_kernel(s->cfg.in_dtype, s->cfg.out_dtype, false);
    size_t nnodes = 0;
    e = hipGraphGetNodes(g, nullptr, &nnodes);
    if (e != hipSuccess) return hip_error(e, "hipGraphGetNodes");
    std::vector<hipGraphNode_t> nodes(nnodes);
    e = hipGraphGetNodes(g, nodes.data(), &nnodes);
    if (e != hipSuccess) return hip_error(e, "hipGraphGetNodes");
    for (hipGraphNode_t n : nodes) {
        hipGraphNodeType type;
        if (hipGraphNodeGetType(n, &type) != hipSuccess || type != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        e = hipGraphKernelNodeGetParams(n, &kp);
        if (e != hipSuccess) return hip_error(e, "hipGraphKernelNodeGetParams");
        if (kp.func == main_fn) {
            sl.main_node = n;
            sl.main_params = kp;
        }
    }
    if (!sl.main_node) return set_error(FOV_EHIP, "captured batch graph has no main kernel node");
    e = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    return FOV_OK;
}

// Launch a batch on a slot; on failure the caller completes it with the error.
// `ready` holds the producer events of the batch's frames that have one.
fov_status launch_batch(ServerImpl* s, Slot& sl, const std::vector<FrameDesc>& frames, int nfrag,
                        const std::vector<hipEvent_t>& ready) {
    if (s->fake_mode()) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fake_q.push_back({now_s() + s->cfg.test_fake_device_us * 1e-6, &sl});
        s->fake_cv.notify_all();
        return FOV_OK;
    }
    for (hipEvent_t ev : ready) {
        hipError_t e = hipStreamWaitEvent(sl.run, ev, 0);
        if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent(ready)");
    }
    if (s->cfg.use_graph) {
        char* h = static_cast<char*>(sl.host);
        BatchHeader hdr{(int32_t)frames.size(), nfrag, queue_slots(nfrag, s->r_cap), 0};
        std::memcpy(h, &hdr, sizeof(hdr));
        std::memcpy(h + sizeof(BatchHeader), frames.data(), frames.size() * sizeof(FrameDesc));
        int32_t* pre = reinterpret_cast<int32_t*>(h + sizeof(BatchHeader) + (size_t)s->cfg.max_batch_frames * sizeof(FrameDesc));
        int32_t acc = 0;
        for (size_t i = 0; i < frames.size(); ++i) {
            pre[i] = acc;
            acc += frames[i].p.nbx * frames[i].nby;
        }
        pre[frames.size()] = acc;
        sl.main_params.gridDim = dim3((unsigned)hdr.nslots);
        hipError_t e = hipGraphExecKernelNodeSetParams(sl.exec, sl.main_node, &sl.main_params);
        if (e != hipSuccess) return hip_error(e, "hipGraphExecKernelNodeSetParams");
        e = hipGraphLaunch(sl.exec, sl.run);
        if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
        return FOV_OK;
    }
    fov_status st = run_forward(frames, s->cfg.in_dtype, s->cfg.out_dtype, sl.run);
    if (st != FOV_OK) return st;
    hipError_t e = hipLaunchHostFunc(sl.run, on_batch_done, &sl);
    if (e != hipSuccess) return hip_error(e, "hipLaunchHostFunc");
    return FOV_OK;
}

// Admit what the budget allows (FIFO) and, if a stream is free, launch
// everything admitted (up to the batch limits) on it.  Called and returns with
// lk held; the lock is released around the launch itself.  True if a batch
// was launched.
bool dispatch_once(ServerImpl* s, std::unique_lock<std::mutex>& lk) {
    while (!s->pending.empty()) {
        Req& r = s->reqs[s->pending.front()];
        if (s->inflight_bytes + r.bytes > s->cfg.hbm_budget_bytes) break;
        s->inflight_bytes += r.bytes;
        r.t.t_admit = now_s();
        s->admitted.push_back(s->pending.front());
        s->pending.pop_front();
    }
    Slot* free_slot = nullptr;
    for (Slot& sl : s->slots)
        if (!sl.busy) {
            free_slot = &sl;
            break;
        }
    if (!free_slot || s->admitted.empty()) return false;
    std::vector<uint64_t> ids;
    std::vector<FrameDesc> frames;
    std::vector<hipEvent_t> ready;
    int nfrag = 0;
    size_t bytes = 0;
    while (!s->admitted.empty() && (int)ids.size() < s->cfg.max_batch_frames) {
        Req& r = s->reqs[s->admitted.front()];
        if (!ids.empty() && nfrag + r.nfrag > s->cfg.max_fragments) break;
        ids.push_back(s->admitted.front());
        frames.push_back(make_frame_desc(r.in, r.out, 0, r.p));
        if (r.ready) ready.push_back(r.ready);
        nfrag += r.nfrag;
        bytes += r.bytes;
        s->admitted.pop_front();
    }
    const double t = now_s();
    for (uint64_t id : ids) {
        Req& r = s->reqs[id];
        r.t.t_launch = t;
        r.t.batch_frames = (int32_t)ids.size();
    }
    ++s->batches;
    free_slot->busy = true;
    free_slot->tickets = ids;
    free_slot->bytes = bytes;
    free_slot->status =
        (s->cfg.test_fail_every > 0 && s->batches % (uint64_t)s->cfg.test_fail_every == 0) ? FOV_EHIP : FOV_OK;
    lk.unlock();
    const fov_status st = launch_batch(s, *free_slot, frames, nfrag, ready);
    if (st != FOV_OK) {
        free_slot->status = st;
        on_batch_done(free_slot);
    }
    lk.lock();
    return true;
}

void scheduler_loop(ServerImpl* s) {
    if (!s->fake_mode()) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (dispatch_once(s, lk)) continue;
        if (s->closing && s->pending.empty() && s->admitted.empty() && s->busy_slots() == 0) break;
        s->cv.wait(lk);
    }
}

fov_status validate_cfg(const fov_server_cfg& c) {
    if (c.hbm_budget_bytes == 0) return set_error(FOV_EINVAL, "hbm_budget_bytes must be > 0");
    if (c.max_batch_frames < 1 || c.max_batch_frames > 4096) return set_error(FOV_EINVAL, "max_batch_frames in 1..4096");
    if (c.max_inflight_batches < 1 || c.max_inflight_batches > 8)
        return set_error(FOV_EINVAL, "max_inflight_batches in 1..8");
    if (c.max_requests < 1) return set_error(FOV_EINVAL, "max_requests must be >= 1");
    const bool ok = (c.in_dtype == FOV_U8 && (c.out_dtype == FOV_U8 || c.out_dtype == FOV_F32)) ||
                    (c.in_dtype == FOV_F32 && c.out_dtype == FOV_F32) || (c.in_dtype == FOV_F64 && c.out_dtype == FOV_F64);
    if (!ok) return set_error(FOV_EDTYPE, "unsupported dtype pair");
    if (c.max_fragments < 1 || c.max_fragments > (1 << 24)) return set_error(FOV_EINVAL, "max_fragments in 1..2^24");
    if (c.max_block < 1 || c.max_block > kMaxBlock) return set_error(FOV_EINVAL, "max_block in 1..64");
    if (!(c.max_sigma >= 0) || c.max_sigma > 1000) return set_error(FOV_EINVAL, "max_sigma in 0..1000");
    if (c.test_fake_device_us < 0 || c.test_fail_every < 0 || (c.shared_stream != 0 && c.shared_stream != 1))
        return set_error(FOV_EINVAL, "bad test hook or shared_stream");
    return FOV_OK;
}

void release(ServerImpl* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
        if (sl.graph) (void)hipGraphDestroy(sl.graph);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}

}  // namespace
}  // namespace fov

namespace fov {
namespace {
void store_now(void* p) { *static_cast<double*>(p) = now_s(); }
}  // namespace
}  // namespace fov

extern "C" {

double foveate_now(void) { return now_s(); }

fov_status foveate_stream_timestamp(void* stream, double* out) {
    if (!out) return set_error(FOV_EINVAL, "out is NULL");
    hipError_t e = hipLaunchHostFunc((hipStream_t)stream, store_now, out);
    if (e != hipSuccess) return hip_error(e, "hipLaunchHostFunc");
    return FOV_OK;
}

fov_status foveate_server_create(const fov_server_cfg* cfg, fov_server** out) {
    if (!cfg || !out) return set_error(FOV_EINVAL, "NULL argument");
    *out = nullptr;
    fov_status st = validate_cfg(*cfg);
    if (st != FOV_OK) return st;
    ServerImpl* s = new ServerImpl();
    s->cfg = *cfg;
    s->r_cap = radius_of(cfg->max_sigma);
    s->slots.resize(cfg->max_inflight_batches);
    for (int i = 0; i < cfg->max_inflight_batches; ++i) {
        s->slots[i].owner = s;
        s->slots[i].index = i;
    }
    if (!s->fake_mode()) {
        hipError_t e = hipGetDevice(&s->device);
        if (e != hipSuccess) {
            release(s);
            return hip_error(e, "hipGetDevice");
        }
        for (Slot& sl : s->slots) {
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                release(s);
                return hip_error(e, "hipStreamCreate");
            }
            if (cfg->use_graph && (st = build_graph(s, sl)) != FOV_OK) {
                release(s);
                return st;
            }
            sl.run = cfg->shared_stream ? s->slots[0].stream : sl.stream;
        }
    } else {
        s->fake = std::thread(fake_device_loop, s);
    }
    s->sched = std::thread(scheduler_loop, s);
    fov_server* h = new fov_server{s};
    *out = h;
    return FOV_OK;
}

fov_status foveate_submit(fov_server* srv, const fov_tensor* in, const fov_tensor* out, const fov_params* p,
                          void* ready, uint64_t* ticket) {
    if (!srv || !ticket) return set_error(FOV_EINVAL, "NULL argument");
    ServerImpl* s = srv->impl;
    bool empty = false;
    fov_status st = prepare(in, out, p, 1, false, &empty);
    if (st != FOV_OK) return st;
    if (in->dtype != s->cfg.in_dtype || out->dtype != s->cfg.out_dtype)
        return set_error(FOV_EDTYPE, "request dtypes differ from the server's");
    Req r;
    r.in = *in;
    r.out = *out;
    r.p = *p;
    r.ready = static_cast<hipEvent_t>(ready);
    if (!empty) {
        if (in->n != 1) return set_error(FOV_EINVAL, "a request holds one frame (n == 1)");
        if (p->block > s->cfg.max_block) return set_error(FOV_EINVAL, "block exceeds the server's max_block");
        const FrameParams f = to_frame(*p, in->h, in->w);
        r.nfrag = f.nbx * grid_extent(in->h, p->origin_y, p->block);
        if (r.nfrag > s->cfg.max_fragments) return set_error(FOV_EINVAL, "frame has more fragments than max_fragments");
        if (frame_r_max(f, in->h) > s->r_cap) return set_error(FOV_ERANGE, "a fragment's sigma exceeds max_sigma");
        r.bytes = view_bytes(*in) + view_bytes(*out);
        if (r.bytes > s->cfg.hbm_budget_bytes) return set_error(FOV_EINVAL, "frame larger than the HBM budget");
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->closing) return set_error(FOV_ECLOSED, "server is shutting down");
    if ((int64_t)s->reqs.size() >= s->cfg.max_requests) return set_error(FOV_EAGAIN, "request table full");
    const uint64_t id = s->next_ticket++;
    r.t.t_submit = now_s();
    if (empty) {
        r.done = true;
        r.t.t_admit = r.t.t_launch = r.t.t_done = r.t.t_submit;
    }
    s->reqs.emplace(id, r);
    *ticket = id;
    if (empty) return FOV_OK;
    s->pending.push_back(id);
    // Fast path: with a stream free and nothing queued ahead, the calling
    // thread admits and launches right away (no hand-off to the scheduler);
    // otherwise the scheduler batches the frame with whatever else waits.
    if (s->pending.size() == 1 && s->admitted.empty()) {
        int prev = -1;
        if (!s->fake_mode() && hipGetDevice(&prev) == hipSuccess && prev != s->device) (void)hipSetDevice(s->device);
        (void)dispatch_once(s, lk);
        if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
    }
    s->cv.notify_all();
    return FOV_OK;
}

fov_status foveate_poll(fov_server* srv, uint64_t ticket, int32_t* done, fov_timing* t) {
    if (!srv || !done) return set_error(FOV_EINVAL, "NULL argument");
    ServerImpl* s = srv->impl;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(FOV_ENOTICKET, "unknown or retired ticket");
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return FOV_OK;
    if (t) *t = it->second.t;
    const fov_status st = (fov_status)it->second.t.status;
    s->reqs.erase(it);
    if (st != FOV_OK) return set_error(st, "the frame's batch failed");
    return FOV_OK;
}

fov_status foveate_server_drain(fov_server* srv) {
    if (!srv) return set_error(FOV_EINVAL, "NULL argument");
    ServerImpl* s = srv->impl;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->pending.empty() && s->admitted.empty() && s->busy_slots() == 0; });
    return FOV_OK;
}

fov_status foveate_server_destroy(fov_server* srv) {
    if (!srv) return set_error(FOV_EINVAL, "NULL argument");
    ServerImpl* s = srv->impl;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing = true;
        s->cv.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fake_stop = true;
        s->fake_cv.notify_all();
    }
    if (s->fake.joinable()) s->fake.join();
    release(s);
    delete srv;
    return FOV_OK;
}

}  // extern "C"
