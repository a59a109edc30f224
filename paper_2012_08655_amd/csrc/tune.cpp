// Launch tuning of the forward kernel: the tuning cache, the thread's forced
// configuration, and the autotuner that times every configuration that fits
// and caches the fastest for the call's workload class.
//
// The choices (output tile split, strip height, dispatch mode, merged pairs of
// capped fragments, per-channel items of small radii) change how fragments map
// onto workgroups, never the
// arithmetic of an output pixel, so the cache can be consulted freely: results
// are the same bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host.h"

namespace fov {
namespace {

struct TuneKey {
    std::string arch;
    int cus, in_dtype, out_dtype, c, bmax, r_bits, frag_bits, frames_class;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, cus, in_dtype, out_dtype, c, bmax, r_bits, frag_bits, frames_class) <
               std::tie(o.arch, o.cus, o.in_dtype, o.out_dtype, o.c, o.bmax, o.r_bits, o.frag_bits, o.frames_class);
    }
};

struct TuneEntry {
    LaunchCfg cfg;
    float us = 0.0f;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
thread_local bool g_forced_on = false;
thread_local LaunchCfg g_forced;

int bit_length(int64_t v) {
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

TuneKey make_key(const DeviceInfo& dev, int nframes, int in_dtype, int out_dtype, const CallShape& cs) {
    TuneKey k;
    k.arch = dev.arch;
    // the arch string has no blanks in practice; keep the text format safe anyway
    std::replace(k.arch.begin(), k.arch.end(), ' ', '_');
    if (k.arch.empty()) k.arch = "unknown";
    k.cus = dev.cus;
    k.in_dtype = in_dtype;
    k.out_dtype = out_dtype;
    k.c = cs.c;
    k.bmax = cs.bmax;
    k.r_bits = bit_length(cs.r_cap);
    k.frag_bits = bit_length(cs.nfrag);
    k.frames_class = nframes <= 1 ? 0 : (nframes <= kArgFrames ? 1 : 2);
    return k;
}

LaunchCfg default_cfg() {
    LaunchCfg c;
    c.split_log2 = 0;
    c.strip_rows = choose_strip_rows();
    c.persistent = dispatch_persistent();
    c.merge = -1;
    c.chan_split = -1;
    return c;
}

bool valid_public(const fov_tuning& t) {
    return (t.split == 1 || t.split == 2 || t.split == 4) &&
           (t.strip_rows == 16 || t.strip_rows == 32 || t.strip_rows == 64) &&
           (t.persistent == 0 || t.persistent == 1) && (t.merge == 0 || t.merge == 1) &&
           (t.chan_split == 0 || t.chan_split == 1) && !(t.merge == 1 && t.split != 1) &&
           !(t.chan_split == 1 && t.split != 1);
}

LaunchCfg from_public(const fov_tuning& t) {
    LaunchCfg c;
    c.split_log2 = t.split == 4 ? 2 : (t.split == 2 ? 1 : 0);
    c.strip_rows = t.strip_rows;
    c.persistent = t.persistent != 0;
    c.merge = t.merge;
    c.chan_split = t.chan_split;
    return c;
}

fov_tuning to_public(const LaunchCfg& c, float us) {
    fov_tuning t;
    t.split = 1 << c.split_log2;
    t.strip_rows = c.strip_rows;
    t.persistent = c.persistent ? 1 : 0;
    t.merge = c.merge > 0 ? 1 : 0;
    t.chan_split = c.chan_split != 0 ? 1 : 0;
    t.time_us = us;
    return t;
}

// Every configuration that fits the device's LDS for this call.  Strip heights
// at or above the tallest padded tile behave alike; only the smallest such is
// kept.  Splits stop at tiles of 8 pixels, and calls with enough fragments to
// fill the chip several times over are not split (more halo work for nothing;
// their work-item counts also make the single-workgroup order pass slow).
constexpr int64_t kSplitMaxFragments = 4096;
std::vector<LaunchCfg> candidates(const DeviceInfo& dev, int in_dtype, const CallShape& cs) {
    std::vector<LaunchCfg> out;
    for (int L = 0; L <= 2; ++L) {
        const int tile = (cs.bmax + (1 << L) - 1) >> L;
        if (L > 0 && (tile < 8 || tile == cs.bmax || cs.nfrag >= kSplitMaxFragments)) break;
        for (int merge : {0, 1}) {
            if (merge && (L > 0 || cs.r_cap == 0)) continue;
            const int th = merge ? 2 * tile : tile;
            const int rows = forward_tile_rows(cs.r_cap, th);
            int prev = -1;
            for (int sr : {16, 32, 64}) {
                const int eff = std::min(sr, rows);
                if (eff == prev) continue;
                prev = eff;
                if (forward_lds_bytes(in_dtype, cs.r_cap, tile, th, sr) + 64 > dev.lds_limit) continue;
                for (bool persist : {false, true})
                    for (int chan : {0, 1}) {
                        if (chan && (L > 0 || cs.c < 2 || cs.c > 16)) continue;
                        LaunchCfg c;
                        c.split_log2 = L;
                        c.strip_rows = sr;
                        c.persistent = persist;
                        c.merge = merge;
                        c.chan_split = chan;
                        out.push_back(c);
                    }
            }
        }
    }
    return out;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

fov_status autotune_frames(const std::vector<FrameDesc>& frames, int in_dtype, int out_dtype, int reps,
                           hipStream_t stream, fov_tuning* best_out) {
    const DeviceInfo* dev = nullptr;
    fov_status s = device_info(&dev);
    if (s != FOV_OK) return s;
    if (reps < 0 || reps > 1000) return set_error(FOV_EINVAL, "reps must be in 0..1000");
    if (reps == 0) reps = 5;
    const CallShape cs = call_shape(frames.data(), (int)frames.size());
    const std::vector<LaunchCfg> cands = candidates(*dev, in_dtype, cs);
    if (cands.empty()) {
        // no configuration fits: let a plain call report the LDS error
        const LaunchCfg d = default_cfg();
        return run_forward(frames, in_dtype, out_dtype, stream, &d, false);
    }
    std::vector<EventPair> ev(reps);
    auto release = [&]() {
        for (EventPair& p : ev) {
            if (p.a) (void)hipEventDestroy(p.a);
            if (p.b) (void)hipEventDestroy(p.b);
        }
    };
    for (EventPair& p : ev) {
        hipError_t e = hipEventCreate(&p.a);
        if (e == hipSuccess) e = hipEventCreate(&p.b);
        if (e != hipSuccess) {
            release();
            return hip_error(e, "hipEventCreate(autotune)");
        }
    }
    float best_us = 0.0f;
    int best = -1;
    std::vector<float> t(reps);
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        const LaunchCfg& c = cands[ci];
        s = run_forward(frames, in_dtype, out_dtype, stream, &c, false);  // warm-up (first-use setup)
        for (int i = 0; s == FOV_OK && i < reps; ++i) {
            hipError_t e = hipEventRecord(ev[i].a, stream);
            if (e != hipSuccess) s = hip_error(e, "hipEventRecord(autotune)");
            if (s == FOV_OK) s = run_forward(frames, in_dtype, out_dtype, stream, &c, false);
            if (s == FOV_OK && (e = hipEventRecord(ev[i].b, stream)) != hipSuccess)
                s = hip_error(e, "hipEventRecord(autotune)");
        }
        for (int i = 0; s == FOV_OK && i < reps; ++i) {
            hipError_t e = hipEventSynchronize(ev[i].b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[i], ev[i].a, ev[i].b);
            if (e != hipSuccess) s = hip_error(e, "hipEventElapsedTime(autotune)");
        }
        if (s != FOV_OK) {
            release();
            return s;
        }
        std::sort(t.begin(), t.end());
        const float med = 1000.0f * t[reps / 2];
        if (best < 0 || med < best_us) {
            best = (int)ci;
            best_us = med;
        }
    }
    release();
    const LaunchCfg& bc = cands[best];
    s = run_forward(frames, in_dtype, out_dtype, stream, &bc, false);
    if (s != FOV_OK) return s;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize(autotune)");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        TuneEntry& te = g_tune[make_key(*dev, (int)frames.size(), in_dtype, out_dtype, cs)];
        te.cfg = bc;
        te.us = best_us;
    }
    if (best_out) *best_out = to_public(bc, best_us);
    return FOV_OK;
}

constexpr const char* kTag = "fov-tune-v3";

}  // namespace

LaunchCfg select_cfg(int nframes, int in_dtype, int out_dtype, const CallShape& cs) {
    if (g_forced_on) return g_forced;
    const DeviceInfo* dev = nullptr;
    if (device_info(&dev) == FOV_OK) {
        const TuneKey k = make_key(*dev, nframes, in_dtype, out_dtype, cs);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(k);
        if (it != g_tune.end()) return it->second.cfg;
    }
    return default_cfg();
}

}  // namespace fov

using namespace fov;

extern "C" {

fov_status foveate_autotune(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                            int32_t reps, void* stream, fov_tuning* best) {
    std::vector<FrameDesc> frames;
    int dt_in = 0, dt_out = 0;
    fov_status s = collect_single(in, out, p, np, &frames, &dt_in, &dt_out);
    if (s != FOV_OK) return s;
    if (frames.empty()) return set_error(FOV_EINVAL, "nothing to tune: the views are empty");
    return autotune_frames(frames, dt_in, dt_out, reps, (hipStream_t)stream, best);
}

fov_status foveate_autotune_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps,
                                  int32_t nframes, int32_t reps, void* stream, fov_tuning* best) {
    std::vector<FrameDesc> frames;
    int dt_in = 0, dt_out = 0;
    fov_status s = collect_batch(ins, outs, ps, nframes, &frames, &dt_in, &dt_out);
    if (s != FOV_OK) return s;
    if (frames.empty()) return set_error(FOV_EINVAL, "nothing to tune: every frame is empty");
    return autotune_frames(frames, dt_in, dt_out, reps, (hipStream_t)stream, best);
}

fov_status foveate_tuning_force(const fov_tuning* t) {
    if (!t) {
        g_forced_on = false;
        return FOV_OK;
    }
    if (!valid_public(*t))
        return set_error(FOV_EINVAL, "split must be 1, 2 or 4, strip_rows 16, 32 or 64, persistent, merge and "
                                     "chan_split 0 or 1 (merge and chan_split with split 1 only)");
    g_forced = from_public(*t);
    g_forced_on = true;
    return FOV_OK;
}

fov_status foveate_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return FOV_OK;
}

fov_status foveate_tuning_count(int32_t* n) {
    if (!n) return set_error(FOV_EINVAL, "n is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *n = (int32_t)g_tune.size();
    return FOV_OK;
}

fov_status foveate_tuning_save(const char* path) {
    if (!path) return set_error(FOV_EINVAL, "path is NULL");
    std::map<TuneKey, TuneEntry> copy;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        copy = g_tune;
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(FOV_EINVAL, std::string("cannot open ") + path + " for writing");
    std::fprintf(f, "# %s arch cus in_dtype out_dtype channels block r_bits frag_bits frames_class : split strip_rows "
                    "persistent merge chan_split time_us\n", kTag);
    for (const auto& kv : copy) {
        const TuneKey& k = kv.first;
        const fov_tuning t = to_public(kv.second.cfg, kv.second.us);
        std::fprintf(f, "%s %s %d %d %d %d %d %d %d %d : %d %d %d %d %d %.3f\n", kTag, k.arch.c_str(), k.cus,
                     k.in_dtype, k.out_dtype, k.c, k.bmax, k.r_bits, k.frag_bits, k.frames_class, t.split,
                     t.strip_rows, t.persistent, t.merge, t.chan_split, (double)t.time_us);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) return set_error(FOV_EINVAL, std::string("error writing ") + path);
    return FOV_OK;
}

fov_status foveate_tuning_load(const char* path) {
    if (!path) return set_error(FOV_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_error(FOV_EINVAL, std::string("cannot open ") + path);
    std::map<TuneKey, TuneEntry> add;
    char line[512];
    int lineno = 0;
    fov_status s = FOV_OK;
    while (std::fgets(line, sizeof(line), f)) {
        ++lineno;
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            s = set_error(FOV_EINVAL, std::string(path) + ":" + std::to_string(lineno) + ": line too long");
            break;
        }
        const char* p = line;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == '\0') continue;
        char tag[32], arch[64];
        TuneKey k;
        fov_tuning t;
        double us = 0.0;
        int used = 0;
        const int got = std::sscanf(p, "%31s %63s %d %d %d %d %d %d %d %d : %d %d %d %d %d %lf %n", tag, arch,
                                    &k.cus, &k.in_dtype, &k.out_dtype, &k.c, &k.bmax, &k.r_bits, &k.frag_bits,
                                    &k.frames_class, &t.split, &t.strip_rows, &t.persistent, &t.merge,
                                    &t.chan_split, &us, &used);
        if (got != 16 || std::strcmp(tag, kTag) != 0 || p[used] != '\0' || !valid_public(t) || k.cus < 1 ||
            k.in_dtype < 0 || k.in_dtype > 2 || k.out_dtype < 0 || k.out_dtype > 2 || k.c < 1 || k.bmax < 1 ||
            k.bmax > kMaxBlock || k.r_bits < 0 || k.r_bits > 31 || k.frag_bits < 0 || k.frag_bits > 62 ||
            k.frames_class < 0 || k.frames_class > 2 || !(us >= 0.0)) {
            s = set_error(FOV_EINVAL, std::string(path) + ":" + std::to_string(lineno) + ": malformed tuning entry");
            break;
        }
        k.arch = arch;
        TuneEntry te;
        te.cfg = from_public(t);
        te.us = (float)us;
        add[k] = te;
    }
    std::fclose(f);
    if (s != FOV_OK) return s;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : add) g_tune[kv.first] = kv.second;
    return FOV_OK;
}

}  // extern "C"
