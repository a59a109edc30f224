// C ABI of libfoveate.so: argument validation, planning on the host for
// launch sizing, and dispatch to the HIP kernels.  Every entry point returns a
// fov_status and never throws.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "adjoint.h"
#include "common.h"
#include "forward.h"
#include "host.h"

namespace fov {

namespace {
thread_local std::string g_last_error;
constexpr int kMaxDevices = 64;
DeviceInfo g_dev[kMaxDevices];
std::mutex g_dev_mu;
}  // namespace

const std::string& last_error() { return g_last_error; }

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

fov_status set_error(fov_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

fov_status hip_error(hipError_t e, const char* what) {
    return set_error(FOV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

fov_status device_info(const DeviceInfo** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(FOV_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo& d = g_dev[dev];
    if (!d.ready) {
        int a = 0, b = 0, cus = 0;
        e = hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return hip_error(e, "hipDeviceGetAttribute(shared per block)");
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
            (void)hipGetLastError();
            b = 0;
        }
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_error(e, "hipDeviceGetAttribute(CU count)");
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_error(e, "hipGetDeviceProperties");
        std::strncpy(d.arch, prop.gcnArchName, sizeof(d.arch) - 1);
        d.lds_limit = (size_t)std::max(a, b);
        d.cus = cus;
        d.ready = true;
    }
    *out = &d;
    return FOV_OK;
}

// Library-owned workspace, one per (device, stream): work queued on one stream
// is ordered, so consecutive calls on that stream may reuse it.  It holds a
// device buffer (plans, queues, frame tables) and a pinned host buffer for
// uploading frame tables.  Both only grow; before a device buffer in use is
// freed the stream is drained, and before the pinned buffer is rewritten the
// previous upload from it is waited for.
namespace {
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
}  // namespace

fov_status workspace(hipStream_t stream, size_t dev_bytes, size_t host_bytes, Workspace** out,
                     std::unique_lock<std::mutex>* hold) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    Workspace* wp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);  // map entries never move or disappear
        wp = &g_ws[{dev, stream}];
    }
    Workspace& w = *wp;
    *hold = std::unique_lock<std::mutex>(w.mu);
    if (w.dev_bytes < dev_bytes) {
        if (w.dev) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize(workspace growth)");
            e = hipFree(w.dev);
            if (e != hipSuccess) return hip_error(e, "hipFree(workspace)");
            w.dev = nullptr;
            w.dev_bytes = 0;
        }
        const size_t nb = std::max(dev_bytes, (size_t)1 << 20);
        e = hipMalloc(&w.dev, nb);
        if (e != hipSuccess) {
            w.dev = nullptr;
            return set_error(FOV_ENOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
        }
        w.dev_bytes = nb;
    }
    if (host_bytes > 0 && w.host_bytes < host_bytes) {
        if (w.host) {
            if (w.upload_pending) {
                e = hipEventSynchronize(w.upload_done);
                if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(upload)");
                w.upload_pending = false;
            }
            e = hipHostFree(w.host);
            if (e != hipSuccess) return hip_error(e, "hipHostFree(staging)");
            w.host = nullptr;
            w.host_bytes = 0;
        }
        const size_t nb = std::max(host_bytes, (size_t)1 << 16);
        e = hipHostMalloc(&w.host, nb, hipHostMallocDefault);
        if (e != hipSuccess) {
            w.host = nullptr;
            return set_error(FOV_ENOMEM, std::string("pinned staging allocation failed: ") + hipGetErrorString(e));
        }
        w.host_bytes = nb;
        if (!w.upload_done) {
            e = hipEventCreateWithFlags(&w.upload_done, hipEventDisableTiming);
            if (e != hipSuccess) return hip_error(e, "hipEventCreate");
        }
    }
    *out = &w;
    return FOV_OK;
}

// Launch attributes of the kernels, per device: dynamic-LDS permission and
// occupancy queries, behind one lock so that concurrent first launches from
// several threads neither race nor pair one size with another's answer.
namespace {
std::mutex g_attr_mu;
std::map<std::pair<int, const void*>, bool> g_lds_set;
std::map<std::tuple<int, const void*, size_t>, int> g_occ;
}  // namespace

fov_status allow_dyn_lds(const void* kern, size_t lds_limit) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (g_lds_set.count({dev, kern})) return FOV_OK;
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, kern);
    if (e != hipSuccess) return hip_error(e, "hipFuncGetAttributes");
    const size_t dyn_max = lds_limit > fa.sharedSizeBytes ? lds_limit - fa.sharedSizeBytes : 0;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_max);
    if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(dynamic LDS)");
    g_lds_set[{dev, kern}] = true;
    return FOV_OK;
}

int occupancy_of(const void* kern, size_t lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    std::lock_guard<std::mutex> lk(g_attr_mu);
    const auto key = std::make_tuple(dev, kern, lds);
    auto it = g_occ.find(key);
    if (it != g_occ.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kThreads, lds) != hipSuccess) {
        (void)hipGetLastError();
        nb = 0;
    }
    g_occ[key] = nb;
    return nb;
}

size_t dtype_size(int dt) {
    switch (dt) {
        case FOV_U8: return 1;
        case FOV_F32: return 4;
        case FOV_F64: return 8;
        default: return 0;
    }
}

bool is_empty(const fov_tensor& t) { return t.n == 0 || t.c == 0 || t.h == 0 || t.w == 0; }

// Largest element offset reachable in the view (strides >= 0).
int64_t max_offset(const fov_tensor& t) {
    return (int64_t)(t.n - 1) * t.sn + (int64_t)(t.c - 1) * t.sc + (int64_t)(t.h - 1) * t.sh +
           (int64_t)(t.w - 1) * t.sw;
}

fov_status check_view(const fov_tensor* t, const char* name, bool is_output) {
    if (!t) return set_error(FOV_EINVAL, std::string(name) + " is NULL");
    if (t->n < 0 || t->c < 0 || t->h < 0 || t->w < 0) return set_error(FOV_EINVAL, std::string(name) + ": negative extent");
    if (dtype_size(t->dtype) == 0) return set_error(FOV_EDTYPE, std::string(name) + ": unknown dtype");
    if (is_empty(*t)) return FOV_OK;
    if (!t->data) return set_error(FOV_EINVAL, std::string(name) + ": data is NULL");
    if (t->sn < 0 || t->sc < 0 || t->sh < 0 || t->sw < 0)
        return set_error(FOV_ELAYOUT, std::string(name) + ": negative stride");
    if ((uintptr_t)t->data % dtype_size(t->dtype) != 0)
        return set_error(FOV_ELAYOUT, std::string(name) + ": misaligned data pointer");
    if (is_output) {
        // Non-overlap: visiting dims by ascending stride, each stride must exceed
        // the span of all smaller dims.
        int64_t ext[4] = {t->n, t->c, t->h, t->w};
        int64_t st[4] = {t->sn, t->sc, t->sh, t->sw};
        int idx[4] = {0, 1, 2, 3};
        std::sort(idx, idx + 4, [&](int a, int b) { return st[a] < st[b]; });
        int64_t span = 0;
        for (int k = 0; k < 4; ++k) {
            int d = idx[k];
            if (ext[d] == 1) continue;
            if (st[d] <= span) return set_error(FOV_ELAYOUT, std::string(name) + ": layout overlaps itself");
            span += (ext[d] - 1) * st[d];
        }
    }
    if (max_offset(*t) > ((int64_t)1 << 40)) return set_error(FOV_EINVAL, std::string(name) + ": view too large");
    if ((int64_t)(t->w - 1) * t->sw >= ((int64_t)1 << 31))
        return set_error(FOV_EINVAL, std::string(name) + ": a row spans more than 2^31 elements");
    return FOV_OK;
}

fov_status check_alias(const fov_tensor& a, const fov_tensor& b) {
    uintptr_t a0 = (uintptr_t)a.data, a1 = a0 + (uintptr_t)(max_offset(a) + 1) * dtype_size(a.dtype);
    uintptr_t b0 = (uintptr_t)b.data, b1 = b0 + (uintptr_t)(max_offset(b) + 1) * dtype_size(b.dtype);
    if (a0 < b1 && b0 < a1) return set_error(FOV_EALIAS, "output memory overlaps input memory");
    return FOV_OK;
}

fov_status check_params(const fov_params& p, int idx) {
    auto bad = [&](const char* what) {
        return set_error(FOV_EINVAL, "params[" + std::to_string(idx) + "]: " + what);
    };
    if (!std::isfinite(p.fix_x) || !std::isfinite(p.fix_y)) return bad("fixation must be finite");
    if (!std::isfinite(p.e0)) return bad("e0 must be finite");
    if (!std::isfinite(p.slope) || p.slope < 0) return bad("slope must be finite and >= 0");
    if (!std::isfinite(p.cap) || p.cap < 0) return bad("cap must be finite and >= 0");
    if (p.block < 1 || p.block > kMaxBlock) return bad("block must be in 1..64");
    if (p.origin_x > 0 || p.origin_x <= -p.block || p.origin_y > 0 || p.origin_y <= -p.block)
        return bad("origin must lie in (-block, 0]");
    if (p.reserved != 0) return bad("reserved must be 0");
    return FOV_OK;
}

FrameParams to_frame(const fov_params& p, int h, int w) {
    FrameParams f;
    f.fix_x = p.fix_x; f.fix_y = p.fix_y; f.e0 = p.e0; f.slope = p.slope; f.cap = p.cap;
    f.block = p.block; f.origin_x = p.origin_x; f.origin_y = p.origin_y;
    f.nbx = grid_extent(w, p.origin_x, p.block);
    f.sigma_map = p.sigma_map;
    (void)h;
    return f;
}

// Largest fragment radius of a frame.  For the eccentricity ramp, distance to
// the fixation is convex over the fragment grid, so its maximum (and hence the
// largest sigma) is reached at one of the four corner fragments.  With a sigma
// map the bound is the cap.
int frame_r_max(const FrameParams& f, int h) {
    if (f.sigma_map) return radius_of(f.cap);
    int nby = grid_extent(h, f.origin_y, f.block);
    int r = 0;
    const int xs[2] = {0, f.nbx - 1}, ys[2] = {0, nby - 1};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) r = std::max(r, radius_of(fragment_sigma_ramp(f, xs[i], ys[j])));
    return r;
}

namespace {
// Per-thread kernel timing (foveate_profile_begin/end): event pairs recorded
// around each main forward kernel while active.
struct Profiler {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    size_t calls = 0;  // forward calls since foveate_profile_begin
    int every = 1;     // record one call in `every`
};
thread_local Profiler g_prof;

void profile_release() {
    for (auto& pr : g_prof.ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    g_prof.ev.clear();
    g_prof.used = 0;
    g_prof.calls = 0;
    g_prof.every = 1;
    g_prof.on = false;
}
}  // namespace

// Dispatch of the main forward kernel: FOV_PERSISTENT=1 selects the
// persistent grid; by default each fragment is its own workgroup (measured
// faster on MI355X for single frames and batches alike).
bool dispatch_persistent() {
    static const bool v = env_int("FOV_PERSISTENT", 0) != 0;
    return v;
}

// Padded-tile rows resident in LDS at once: the kernel's strip height (64
// rows, four rows per lane of a wave) unless FOV_STRIP_ROWS asks for fewer.
int choose_strip_rows() {
    static const int forced = env_int("FOV_STRIP_ROWS", 0);
    const int mx = forward_strip_max();
    return forced > 0 && forced < mx ? forced : mx;
}

// Shared validation of forward/backward arguments.
fov_status prepare(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                          bool backward, bool* empty) {
    fov_status s;
    if ((s = check_view(in, backward ? "grad_out" : "in", false)) != FOV_OK) return s;
    if ((s = check_view(out, backward ? "grad_in" : "out", true)) != FOV_OK) return s;
    if (in->n != out->n || in->c != out->c || in->h != out->h || in->w != out->w)
        return set_error(FOV_EINVAL, "input and output shapes differ");
    if (backward) {
        if (!((in->dtype == FOV_F32 && out->dtype == FOV_F32) || (in->dtype == FOV_F64 && out->dtype == FOV_F64)))
            return set_error(FOV_EDTYPE, "backward supports f32->f32 and f64->f64");
    } else {
        bool ok = (in->dtype == FOV_U8 && (out->dtype == FOV_U8 || out->dtype == FOV_F32)) ||
                  (in->dtype == FOV_F32 && out->dtype == FOV_F32) || (in->dtype == FOV_F64 && out->dtype == FOV_F64);
        if (!ok) return set_error(FOV_EDTYPE, "unsupported dtype pair");
    }
    *empty = is_empty(*in);
    if (*empty) return FOV_OK;
    if ((s = check_alias(*in, *out)) != FOV_OK) return s;
    if (in->dtype == FOV_U8) {
        // 8-bit frames are read through 32-bit buffer offsets
        const int64_t span = (int64_t)(in->c - 1) * in->sc + (int64_t)(in->h - 1) * in->sh + (int64_t)(in->w - 1) * in->sw + 1;
        if (span >= ((int64_t)1 << 31)) return set_error(FOV_EINVAL, "an 8-bit frame may span at most 2^31 - 1 bytes");
    }
    if (!p) return set_error(FOV_EINVAL, "params is NULL");
    if (np != in->n && np != 1) return set_error(FOV_EINVAL, "np must equal n or 1");
    for (int i = 0; i < np; ++i)
        if ((s = check_params(p[i], i)) != FOV_OK) return s;
    return FOV_OK;
}

size_t frame_table_bytes(int nf) { return ((size_t)nf * sizeof(FrameDesc) + (size_t)(nf + 1) * 4 + 255) / 256 * 256; }

// Place a launch's frame descriptors where its kernels read them: in the
// kernel arguments (up to kArgFrames; the plan kernel copies them to dtab) or
// uploaded to dtab from the workspace's pinned buffer.
fov_status stage_frame_table(const FrameDesc* frames, int nf, const int32_t* prefix, Workspace* ws, char* dtab,
                             size_t tbytes, hipStream_t stream, FwdLaunch* a) {
    a->table = reinterpret_cast<FrameDesc*>(dtab);
    a->prefix = reinterpret_cast<int32_t*>(dtab + (size_t)nf * sizeof(FrameDesc));
    if (nf > kArgFrames) {
        if (ws->upload_pending) {
            hipError_t e = hipEventSynchronize(ws->upload_done);
            if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(upload)");
            ws->upload_pending = false;
        }
        char* hst = static_cast<char*>(ws->host);
        std::memcpy(hst, frames, (size_t)nf * sizeof(FrameDesc));
        std::memcpy(hst + (size_t)nf * sizeof(FrameDesc), prefix, (size_t)(nf + 1) * 4);
        hipError_t e = hipMemcpyAsync(dtab, hst, tbytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(frame table)");
        e = hipEventRecord(ws->upload_done, stream);
        if (e != hipSuccess) return hip_error(e, "hipEventRecord(upload)");
        ws->upload_pending = true;
    } else {
        a->from_args = 1;
        for (int i = 0; i < nf; ++i) a->fr[i] = frames[i];
        for (int i = 0; i <= nf; ++i) a->kprefix[i] = prefix[i];
    }
    return FOV_OK;
}

CallShape call_shape(const FrameDesc* frames, int nf) {
    CallShape cs;
    for (int i = 0; i < nf; ++i) {
        const FrameDesc& f = frames[i];
        cs.nfrag += (int64_t)f.p.nbx * f.nby;
        cs.r_cap = std::max(cs.r_cap, frame_r_max(f.p, f.h));
        cs.bmax = std::max(cs.bmax, f.p.block);
        cs.c = std::max(cs.c, f.c);
    }
    return cs;
}

// Launch shape of one forward call over a list of frames (any shapes, one
// dtype pair): counts, radius bound, LDS and scratch sizes; no device work.
fov_status plan_forward(const FrameDesc* frames, int nf, int in_dtype, int out_dtype, const LaunchCfg* cfg_in,
                        ForwardPlan* fp) {
    fov_status s;
    const CallShape cs = call_shape(frames, nf);
    if (cs.r_cap >= kRadiusLimit)
        return set_error(FOV_ERANGE, "a fragment radius exceeds " + std::to_string(kRadiusLimit - 1) +
                                         " pixels; no workgroup can stage its window");
    const DeviceInfo* dev = nullptr;
    if ((s = device_info(&dev)) != FOV_OK) return s;
    const LaunchCfg cfg = cfg_in ? *cfg_in : select_cfg(nf, in_dtype, out_dtype, cs);
    const int L = cfg.split_log2;
    if ((cs.nfrag << (2 * L)) > ((int64_t)1 << 30)) return set_error(FOV_EINVAL, "too many fragments in one call");
    const int r_cap = cs.r_cap;
    const int tile = (cs.bmax + (1 << L) - 1) >> L;
    const int sr = cfg.strip_rows;
    size_t lds = forward_lds_bytes(in_dtype, r_cap, tile, tile, sr);
    // vertical pairs at the cap need tiles twice as tall; by default only when the CU holds as
    // many workgroups with them
    bool merge = cfg.merge != 0 && L == 0 && r_cap > 0;
    if (merge) {
        const size_t lds2 = forward_lds_bytes(in_dtype, r_cap, tile, 2 * tile, sr);
        if (lds2 + 64 > dev->lds_limit ||
            (cfg.merge < 0 && forward_occupancy(in_dtype, out_dtype, lds2) < forward_occupancy(in_dtype, out_dtype, lds)))
            merge = false;
        else
            lds = lds2;
    }
    if (lds + 64 > dev->lds_limit)
        return set_error(FOV_ERANGE, "radius " + std::to_string(r_cap) + " needs " + std::to_string(lds) +
                                         " bytes of LDS; the device allows " + std::to_string(dev->lds_limit));
    const int wsize = in_dtype == FOV_F64 ? 8 : 4;
    FwdLaunch& a = fp->a;
    std::memset(&a, 0, sizeof(a));
    // first fragment of each frame: in the kernel arguments' copy for calls of at most kArgFrames
    // frames (no host allocation), else in the table that launch_planned uploads
    if (nf > kArgFrames) fp->prefix_table.assign(nf + 1, 0);
    int32_t* prefix = nf > kArgFrames ? fp->prefix_table.data() : a.kprefix;
    int64_t total = 0;
    for (int i = 0; i < nf; ++i) {
        prefix[i] = (int32_t)total;
        total += (int64_t)frames[i].p.nbx * frames[i].nby;
    }
    prefix[nf] = (int32_t)total;
    a.nframes = nf;
    a.nfrag = (int32_t)total;
    a.split_log2 = L;
    a.merge = merge ? 1 : 0;
    a.r_cap = r_cap;
    a.strip_rows = sr;
    a.wstride = round_up(2 * r_cap + 1, 16);
    // Fragments of radius <= 2/3 of r_cap become one work item per channel (the latency-bound
    // items at the end of the queue then run their channels side by side).
    const bool chan = cfg.chan_split != 0 && L == 0 && cs.c > 1 && cs.c <= 16 && a.nfrag < (1 << kChanShift);
    const int cs_rmax = chan ? (2 * r_cap) / 3 : -1;
    a.cs_rmax = cs_rmax;
    a.cmax = cs.c;
    a.nslots = cs_rmax >= 0 ? queue_slots_by_channel(a.nfrag, r_cap, cs.c) : queue_slots(a.nfrag << (2 * L), r_cap);
    fp->lds = lds;
    fp->persistent = cfg.persistent;
    fp->pbytes = (plan_bytes(a.nfrag, a.nslots, a.wstride, wsize) + 255) / 256 * 256;
    fp->tbytes = frame_table_bytes(nf);
    fp->lds_limit = dev->lds_limit;
    fp->cus = dev->cus;
    return FOV_OK;
}

// Plan, order and main kernels of a planned call, with its plan workspace at
// `scratch` (at least fp.pbytes + fp.tbytes bytes of device memory).  Frame
// tables of more than kArgFrames frames are uploaded from ws's pinned buffer
// (ws may be NULL for calls of at most kArgFrames frames).
fov_status launch_planned(const FrameDesc* frames, int nf, int in_dtype, int out_dtype, ForwardPlan& fp,
                          void* scratch, Workspace* ws, hipStream_t stream, bool profile) {
    fov_status s;
    FwdLaunch& a = fp.a;
    const PlanBuffers plan = carve_plan(scratch, a.nfrag, a.nslots);
    if ((s = stage_frame_table(frames, nf, fp.prefix(), ws, static_cast<char*>(scratch) + fp.pbytes,
                               fp.tbytes, stream, &a)) != FOV_OK)
        return s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile && g_prof.on && g_prof.calls++ % g_prof.every == 0 && g_prof.used < g_prof.ev.size()) {
        e0 = g_prof.ev[g_prof.used].first;
        e1 = g_prof.ev[g_prof.used].second;
        ++g_prof.used;
    }
    return launch_forward(a, in_dtype, out_dtype, fp.lds, plan, stream, fp.lds_limit, fp.cus, fp.persistent, e0, e1);
}

// One forward launch over a list of frames (any shapes, one dtype pair), its
// plan workspace in the library's per-(device, stream) workspace.  Up to
// kArgFrames descriptors travel in the kernel arguments; more are uploaded
// as a device table from pinned memory.
fov_status run_forward(const std::vector<FrameDesc>& frames, int in_dtype, int out_dtype, hipStream_t stream,
                       const LaunchCfg* cfg_in, bool profile) {
    if (frames.empty()) return FOV_OK;
    fov_status s;
    ForwardPlan fp;
    if ((s = plan_forward(frames.data(), (int)frames.size(), in_dtype, out_dtype, cfg_in, &fp)) != FOV_OK) return s;
    const bool upload = (int)frames.size() > kArgFrames;
    Workspace* ws = nullptr;
    std::unique_lock<std::mutex> hold;
    if ((s = workspace(stream, fp.pbytes + fp.tbytes, upload ? fp.tbytes : 0, &ws, &hold)) != FOV_OK) return s;
    return launch_planned(frames.data(), (int)frames.size(), in_dtype, out_dtype, fp, ws->dev, ws, stream, profile);
}

// Scratch of the adjoint's horizontal transposes, per launch: frames are
// processed in groups whose scratch stays below this (one frame at least).
constexpr size_t kAdjScratchMax = (size_t)256 << 20;

// Adjoint of one frame group on `stream`: transposed windows, then the per-tile sums.
fov_status run_backward_group(const FrameDesc* frames, int nf, int dtype, hipStream_t stream) {
    fov_status s;
    const DeviceInfo* dev = nullptr;
    if ((s = device_info(&dev)) != FOV_OK) return s;
    const CallShape cs = call_shape(frames, nf);
    const int es = dtype == FOV_F64 ? 8 : 4;
    const AdjShape sh = adjoint_shape(es, cs.r_cap, cs.bmax, cs.c);
    std::vector<int32_t> prefix(nf + 1);
    int64_t total = 0;
    for (int i = 0; i < nf; ++i) {
        prefix[i] = (int32_t)total;
        total += (int64_t)frames[i].p.nbx * frames[i].nby;
    }
    prefix[nf] = (int32_t)total;
    if (total > ((int64_t)1 << 30)) return set_error(FOV_EINVAL, "too many fragments in one call");
    FwdLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.nframes = nf;
    a.nfrag = (int32_t)total;
    a.r_cap = cs.r_cap;
    const size_t f4 = ((size_t)a.nfrag * 4 + 255) / 256 * 256;
    const size_t tbytes = frame_table_bytes(nf);
    const size_t sbytes = adjoint_scratch_elems(sh, a.nfrag) * es;
    Workspace* ws = nullptr;
    std::unique_lock<std::mutex> hold;
    if ((s = workspace(stream, f4 + tbytes + sbytes, nf > kArgFrames ? tbytes : 0, &ws, &hold)) != FOV_OK) return s;
    char* base = static_cast<char*>(ws->dev);
    int32_t* radius = reinterpret_cast<int32_t*>(base);
    char* dtab = base + f4;
    void* scratch = dtab + tbytes;
    if ((s = stage_frame_table(frames, nf, prefix.data(), ws, dtab, tbytes, stream, &a)) != FOV_OK) return s;
    return launch_adjoint(a, sh, es, radius, scratch, stream, dev->lds_limit);
}

fov_status run_backward(const fov_tensor* go, const fov_tensor* gi, const fov_params* p, int32_t np,
                        hipStream_t stream) {
    std::vector<FrameDesc> frames;
    frames.reserve(go->n);
    for (int i = 0; i < go->n; ++i) frames.push_back(make_frame_desc(*go, *gi, i, p[np == 1 ? 0 : i]));
    if (call_shape(frames.data(), (int)frames.size()).r_cap >= kRadiusLimit)
        return set_error(FOV_ERANGE, "a fragment radius exceeds " + std::to_string(kRadiusLimit - 1) +
                                         " pixels; no workgroup can stage its window");
    const int es = go->dtype == FOV_F64 ? 8 : 4;
    size_t f0 = 0;
    while (f0 < frames.size()) {
        size_t f1 = f0 + 1;
        CallShape cs = call_shape(&frames[f0], 1);
        while (f1 < frames.size()) {
            const CallShape one = call_shape(&frames[f1], 1);
            CallShape m = cs;
            m.r_cap = std::max(m.r_cap, one.r_cap);
            m.bmax = std::max(m.bmax, one.bmax);
            m.c = std::max(m.c, one.c);
            m.nfrag += one.nfrag;
            const AdjShape sh = adjoint_shape(es, m.r_cap, m.bmax, m.c);
            if (m.nfrag > (1 << 30) || adjoint_scratch_elems(sh, (int)m.nfrag) * es > kAdjScratchMax) break;
            cs = m;
            ++f1;
        }
        fov_status s = run_backward_group(frames.data() + f0, (int)(f1 - f0), go->dtype, stream);
        if (s != FOV_OK) return s;
        f0 = f1;
    }
    return FOV_OK;
}

FrameDesc make_frame_desc(const fov_tensor& in, const fov_tensor& out, int n, const fov_params& p) {
    const size_t ei = dtype_size(in.dtype), eo = dtype_size(out.dtype);
    FrameDesc d;
    d.in = static_cast<const char*>(in.data) + (size_t)n * in.sn * ei;
    d.out = static_cast<char*>(out.data) + (size_t)n * out.sn * eo;
    d.isc = in.sc; d.ish = in.sh; d.isw = in.sw;
    d.osc = out.sc; d.osh = out.sh; d.osw = out.sw;
    d.c = in.c; d.h = in.h; d.w = in.w;
    d.p = to_frame(p, in.h, in.w);
    d.nby = grid_extent(in.h, p.origin_y, p.block);
    return d;
}

fov_status collect_single(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                          std::vector<FrameDesc>* frames, int* dt_in, int* dt_out) {
    bool empty = false;
    fov_status s = prepare(in, out, p, np, false, &empty);
    frames->clear();
    if (s != FOV_OK || empty) return s;
    frames->reserve(in->n);
    for (int i = 0; i < in->n; ++i) frames->push_back(make_frame_desc(*in, *out, i, p[np == 1 ? 0 : i]));
    *dt_in = in->dtype;
    *dt_out = out->dtype;
    return FOV_OK;
}

fov_status collect_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps, int32_t nframes,
                         std::vector<FrameDesc>* frames, int* dt_in, int* dt_out) {
    frames->clear();
    if (nframes < 0) return set_error(FOV_EINVAL, "nframes < 0");
    if (nframes == 0) return FOV_OK;
    if (!ins || !outs || !ps) return set_error(FOV_EINVAL, "NULL argument");
    frames->reserve(nframes);
    *dt_in = *dt_out = -1;
    for (int i = 0; i < nframes; ++i) {
        bool empty = false;
        fov_status s = prepare(&ins[i], &outs[i], &ps[i], 1, false, &empty);
        if (s != FOV_OK) return set_error(s, "frame " + std::to_string(i) + ": " + last_error());
        if (empty) continue;
        if (ins[i].n != 1) return set_error(FOV_EINVAL, "frame " + std::to_string(i) + ": each view must hold one frame");
        if (*dt_in < 0) { *dt_in = ins[i].dtype; *dt_out = outs[i].dtype; }
        if (ins[i].dtype != *dt_in || outs[i].dtype != *dt_out)
            return set_error(FOV_EDTYPE, "all frames of a batch must share one dtype pair");
        frames->push_back(make_frame_desc(ins[i], outs[i], 0, ps[i]));
    }
    // outputs of different frames must not overlap inputs of others either
    for (int i = 0; i < nframes; ++i)
        for (int j = 0; j < nframes; ++j) {
            if (i == j || is_empty(ins[j]) || is_empty(outs[i])) continue;
            fov_status s = check_alias(ins[j], outs[i]);
            if (s != FOV_OK) return set_error(s, "output of frame " + std::to_string(i) + " overlaps input of frame " + std::to_string(j));
            if (j < i) {
                s = check_alias(outs[j], outs[i]);
                if (s != FOV_OK) return set_error(s, "outputs of frames " + std::to_string(j) + " and " + std::to_string(i) + " overlap");
            }
        }
    return FOV_OK;
}

}  // namespace fov

using namespace fov;

extern "C" {

const char* foveate_last_error(void) { return g_last_error.c_str(); }

const char* foveate_version(void) { return "libfoveate 0.1 (gfx950)"; }

fov_status foveate_profile_begin(int32_t capacity) {
    if (capacity < 1 || capacity > (1 << 20)) return set_error(FOV_EINVAL, "capacity must be in 1..2^20");
    profile_release();
    g_prof.ev.reserve(capacity);
    for (int i = 0; i < capacity; ++i) {
        hipEvent_t a = nullptr, b = nullptr;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            profile_release();
            return hip_error(e, "hipEventCreate(profile)");
        }
        g_prof.ev.emplace_back(a, b);
    }
    g_prof.on = true;
    return FOV_OK;
}

fov_status foveate_profile_every(int32_t every) {
    if (every < 1) return set_error(FOV_EINVAL, "every must be at least 1");
    if (!g_prof.on) return set_error(FOV_EINVAL, "profiling was not started");
    g_prof.every = every;
    return FOV_OK;
}

fov_status foveate_profile_end(float* ms, int32_t capacity, int32_t* count) {
    if (!count) return set_error(FOV_EINVAL, "count is NULL");
    *count = 0;
    if (!g_prof.on) return set_error(FOV_EINVAL, "profiling was not started");
    const int n = (int)std::min(g_prof.used, (size_t)std::max(capacity, 0));
    for (int i = 0; i < n; ++i) {
        hipError_t e = hipEventSynchronize(g_prof.ev[i].second);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, g_prof.ev[i].first, g_prof.ev[i].second);
        if (e != hipSuccess) {
            profile_release();
            return hip_error(e, "hipEventElapsedTime(profile)");
        }
        if (ms) ms[i] = t;
    }
    *count = n;
    profile_release();
    return FOV_OK;
}

fov_status foveate_grid(int32_t h, int32_t w, const fov_params* p, int32_t* nbx, int32_t* nby) {
    if (!p || !nbx || !nby) return set_error(FOV_EINVAL, "NULL argument");
    if (h < 1 || w < 1) return set_error(FOV_EINVAL, "frame must be at least 1x1");
    fov_status s = check_params(*p, 0);
    if (s != FOV_OK) return s;
    *nbx = grid_extent(w, p->origin_x, p->block);
    *nby = grid_extent(h, p->origin_y, p->block);
    return FOV_OK;
}

fov_status foveate_csf_params(int32_t h, int32_t w, double e_corner_deg, double f_max_cpd, double cap,
                              fov_params* p) {
    if (!p) return set_error(FOV_EINVAL, "p is NULL");
    if (h < 1 || w < 1 || (h == 1 && w == 1)) return set_error(FOV_EINVAL, "frame must have at least two pixels");
    if (!std::isfinite(e_corner_deg) || e_corner_deg <= 0) return set_error(FOV_EINVAL, "e_corner must be > 0");
    if (!std::isfinite(f_max_cpd) || !std::isfinite(cap) || cap <= 0)
        return set_error(FOV_EINVAL, "f_max must be finite and cap > 0");
    // constants of the contrast-threshold model the paper adopts (Eq. 2)
    const double ct0 = 1.0 / 64.0, alpha = 0.106, e2 = 2.3;
    const double ln_inv_ct0 = std::log(1.0 / ct0);
    const double f_max = f_max_cpd > 0 ? f_max_cpd : ln_inv_ct0 / alpha;  // f_c_deg at e = 0
    const double hx = 0.5 * (w - 1), hy = 0.5 * (h - 1);
    const double d_corner = std::sqrt(hx * hx + hy * hy);
    // sigma(d) = k (e_corner d / d_corner + e2) = slope (d - e0)
    const double k = f_max * alpha / (M_PI * e2 * ln_inv_ct0);
    p->slope = k * e_corner_deg / d_corner;
    p->e0 = -e2 * d_corner / e_corner_deg;
    p->cap = cap;
    return FOV_OK;
}

fov_status foveate_fragment_shift(double fix_x, double fix_y, int32_t block, int32_t* origin_x,
                                  int32_t* origin_y) {
    if (!origin_x || !origin_y) return set_error(FOV_EINVAL, "NULL argument");
    if (block < 1 || block > kMaxBlock) return set_error(FOV_EINVAL, "block must be in 1..64");
    if (!std::isfinite(fix_x) || !std::isfinite(fix_y) || std::fabs(fix_x) > 1e9 || std::fabs(fix_y) > 1e9)
        return set_error(FOV_EINVAL, "fixation must be finite (|f| <= 1e9)");
    auto origin = [block](double f) {
        const int64_t s = (int64_t)std::floor(f - 0.5 * (block - 1) + 0.5);  // start of the centred fragment
        const int64_t m = ((s % block) + block) % block;
        return (int32_t)(m == 0 ? 0 : m - block);
    };
    *origin_x = origin(fix_x);
    *origin_y = origin(fix_y);
    return FOV_OK;
}

fov_status foveate_plan_host(int32_t h, int32_t w, const fov_params* p, double* sigma_out, int32_t* r_out) {
    int32_t nbx, nby;
    fov_status s = foveate_grid(h, w, p, &nbx, &nby);
    if (s != FOV_OK) return s;
    if (!r_out) return set_error(FOV_EINVAL, "r_out is NULL");
    if (p->sigma_map) return set_error(FOV_EINVAL, "host plan cannot read a device sigma map");
    FrameParams f = to_frame(*p, h, w);
    for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) {
            double sg = fragment_sigma_ramp(f, bx, by);
            if (sigma_out) sigma_out[by * nbx + bx] = sg;
            r_out[by * nbx + bx] = radius_of(sg);
        }
    return FOV_OK;
}

fov_status foveate_plan(int32_t h, int32_t w, const fov_params* p, double* sigma_out, int32_t* r_out, void* stream) {
    int32_t nbx, nby;
    fov_status s = foveate_grid(h, w, p, &nbx, &nby);
    if (s != FOV_OK) return s;
    if (!r_out) return set_error(FOV_EINVAL, "r_out is NULL");
    return launch_plan(to_frame(*p, h, w), nbx * nby, sigma_out, r_out, (hipStream_t)stream);
}

fov_status foveate_forward(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                           void* stream) {
    std::vector<FrameDesc> frames;
    int dt_in = 0, dt_out = 0;
    fov_status s = collect_single(in, out, p, np, &frames, &dt_in, &dt_out);
    if (s != FOV_OK || frames.empty()) return s;
    return run_forward(frames, dt_in, dt_out, (hipStream_t)stream);
}

fov_status foveate_forward_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps,
                                 int32_t nframes, void* stream) {
    std::vector<FrameDesc> frames;
    int dt_in = 0, dt_out = 0;
    fov_status s = collect_batch(ins, outs, ps, nframes, &frames, &dt_in, &dt_out);
    if (s != FOV_OK || frames.empty()) return s;
    return run_forward(frames, dt_in, dt_out, (hipStream_t)stream);
}

fov_status foveate_backward(const fov_tensor* grad_out, const fov_tensor* grad_in, const fov_params* p, int32_t np,
                            void* stream) {
    bool empty = false;
    fov_status s = prepare(grad_out, grad_in, p, np, true, &empty);
    if (s != FOV_OK || empty) return s;
    return run_backward(grad_out, grad_in, p, np, (hipStream_t)stream);
}

}  // extern "C"
