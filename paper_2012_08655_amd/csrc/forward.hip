// Forward block-wise foveation for gfx950.
//
// Two launches per batch of frames on the caller's stream:
//
//  1. fov_plan_kernel — one wavefront per fragment: the fragment's sigma from
//     its midpoint's eccentricity (Sec. 2, Fig. 1), radius r = ceil(3 sigma)
//     and the normalised taps w_k = exp(-k^2/(2 sigma^2)) / sum (Eq. 1 cut at
//     3 sigma, Appendix "Methods"), summed with wavefront shuffles, written to
//     the plan workspace zero-padded to a multiple of 4 taps.
//
//  2. fov_fwd_kernel — one workgroup per output fragment (Alg. 1): the padded
//     tile (fragment plus r on each side, clamp-to-edge) is staged into LDS
//     with row-coalesced loads, 8-bit input kept exact as fp16; a horizontal
//     pass writes the fp32 intermediate into LDS; a vertical pass produces the
//     fragment (Appendix "Workload of the Block", "Shared Memory").  Each
//     thread computes 8 (horizontal) or 4 (vertical) outputs and slides the
//     filter window through registers (the register reuse of Appendix "Data
//     Reuse"); the weights are read with scalar loads and used as SGPR
//     operands of the FMAs.  A fragment with r = 0 is copied.
//
// Every output sums its taps in the same order (k = -r .. r) whatever the
// strip height, so results do not depend on tuning choices.
#include "forward.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace fov {

namespace {

constexpr int kPH = 8;  // outputs per thread, horizontal pass
constexpr int kPV = 4;  // outputs per thread, vertical pass
constexpr int kU = 4;   // taps per register-window step

struct Geom {
    int NP;  // taps padded to a multiple of kU (padding taps have weight 0)
    int G;   // horizontal-pass column groups
    int GV;  // vertical-pass row groups
    int TW;  // staged tile columns
    int TH;  // staged tile rows = intermediate rows
};

__host__ __device__ inline Geom geom(int r, int bw, int bh) {
    Geom g;
    g.NP = round_up(2 * r + 1, kU);
    g.G = (bw + kPH - 1) / kPH;
    g.GV = (bh + kPV - 1) / kPV;
    g.TW = g.G * kPH + g.NP;
    g.TH = g.GV * kPV + g.NP;
    return g;
}

// Tile row pitch in elements: rows start 16 bytes apart modulo 128 bytes, so
// eight lanes reading 16 bytes from eight consecutive rows hit 32 distinct
// LDS banks.
__host__ __device__ inline int tile_pitch(int TW, int es) {
    const int q = 16 / es, m = 128 / es;
    return round_up(TW > q ? TW - q : 1, m) + q;
}

__host__ __device__ inline int inter_pitch(int bmax) { return bmax + 4; }

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// ---- element conversions ----------------------------------------------------------------------
template <typename TS, typename TIn>
__device__ __forceinline__ TS to_stage(TIn v) { return (TS)v; }
template <>
__device__ __forceinline__ _Float16 to_stage<_Float16, uint8_t>(uint8_t v) { return (_Float16)(uint16_t)v; }

template <typename TOut, typename TC>
__device__ __forceinline__ TOut to_out(TC v) { return (TOut)v; }
template <>
__device__ __forceinline__ uint8_t to_out<uint8_t, float>(float v) {
    v = rintf(v);  // round half to even
    v = fminf(fmaxf(v, 0.0f), 255.0f);
    return (uint8_t)v;
}

template <typename TOut, typename TIn>
__device__ __forceinline__ TOut copy_out(TIn v) { return (TOut)v; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---- LDS window loads -------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void load4_row(const T* p, T (&b)[4]) {
    if constexpr (sizeof(T) == 2) {
        // 8-byte load of four halves
        const uint2 u = *reinterpret_cast<const uint2*>(p);
        const _Float16* h = reinterpret_cast<const _Float16*>(&u);
        b[0] = h[0]; b[1] = h[1]; b[2] = h[2]; b[3] = h[3];
    } else if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        b[0] = v.x; b[1] = v.y; b[2] = v.z; b[3] = v.w;
    } else {
        const double2 v0 = *reinterpret_cast<const double2*>(p);
        const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
        b[0] = v0.x; b[1] = v0.y; b[2] = v1.x; b[3] = v1.y;
    }
}

template <int IP, typename T>
__device__ __forceinline__ void load4_col(const T* p, T (&b)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = p[k * IP];
}

// Horizontal step: taps j0..j0+3 on 8 outputs; window = X ++ Y ++ Z[0..2].
template <typename TC, typename TS>
__device__ __forceinline__ void hstep(TC (&acc)[kPH], const TS (&X)[4], const TS (&Y)[4], const TS (&Z)[4],
                                      const TC* __restrict__ w) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const TC wu = w[u];
#pragma unroll
        for (int p = 0; p < kPH; ++p) {
            const int i = p + u;
            const TS v = i < 4 ? X[i] : (i < 8 ? Y[i - 4] : Z[i - 8]);
            acc[p] = fma(wu, (TC)v, acc[p]);
        }
    }
}

// Vertical step: taps j0..j0+3 on 4 outputs; window = X ++ Y[0..2].
template <typename TC>
__device__ __forceinline__ void vstep(TC (&acc)[kPV], const TC (&X)[4], const TC (&Y)[4], const TC* __restrict__ w) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const TC wu = w[u];
#pragma unroll
        for (int p = 0; p < kPV; ++p) {
            const int i = p + u;
            acc[p] = fma(wu, i < 4 ? X[i] : Y[i - 4], acc[p]);
        }
    }
}

// 8 horizontal outputs from a staged row (inputs row[0 .. NP+7]).
template <typename TC, typename TS>
__device__ __forceinline__ void hconv(TC (&acc)[kPH], const TS* row, int NP, const TC* __restrict__ w) {
    TS A[4], B[4], C[4];
    load4_row(row, A);
    load4_row(row + 4, B);
    int j0 = 0;
    for (; j0 + 12 <= NP; j0 += 12) {
        load4_row(row + j0 + 8, C);
        hstep(acc, A, B, C, w + j0);
        load4_row(row + j0 + 12, A);
        hstep(acc, B, C, A, w + j0 + 4);
        load4_row(row + j0 + 16, B);
        hstep(acc, C, A, B, w + j0 + 8);
    }
    const int rem = NP - j0;  // 0, 4 or 8
    if (rem >= 4) {
        load4_row(row + j0 + 8, C);
        hstep(acc, A, B, C, w + j0);
        if (rem == 8) {
            load4_row(row + j0 + 12, A);
            hstep(acc, B, C, A, w + j0 + 4);
        }
    }
}

// 4 vertical outputs from an intermediate column (inputs col[0 .. NP+3] rows).
template <int IP, typename TC>
__device__ __forceinline__ void vconv(TC (&acc)[kPV], const TC* col, int NP, const TC* __restrict__ w) {
    TC A[4], B[4];
    load4_col<IP>(col, A);
    int j0 = 0;
    for (; j0 + 8 <= NP; j0 += 8) {
        load4_col<IP>(col + (j0 + 4) * IP, B);
        vstep(acc, A, B, w + j0);
        load4_col<IP>(col + (j0 + 8) * IP, A);
        vstep(acc, B, A, w + j0 + 4);
    }
    if (j0 < NP) {
        load4_col<IP>(col + (j0 + 4) * IP, B);
        vstep(acc, A, B, w + j0);
    }
}

// Stage padded-tile rows [s0, s0+rows) of one channel into LDS.  Lanes walk
// columns (coalesced along x), waves walk rows; each lane's clamped column
// offset is computed once and added to a wave-uniform row pointer, and loads
// for 8 rows x 2 column chunks are issued before any is consumed.
template <typename TIn, typename TS>
__device__ __forceinline__ void stage_rows(TS* tile, int TP, const TIn* plane, int64_t ish, int64_t isw, int y_first,
                                           int x_first, int s0, int rows, int TW, int h, int w) {
    constexpr int RB = 8, KB = 2, kWaves = kThreads / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k0 = 0; k0 < TW; k0 += 64 * KB) {
        uint32_t coff[KB];
        bool cv[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int tx = k0 + kb * 64 + lane;
            cv[kb] = tx < TW;
            coff[kb] = (uint32_t)clampi(x_first + tx, 0, w - 1) * (uint32_t)isw;
        }
        for (int t0 = wave; t0 < rows; t0 += kWaves * RB) {
            TIn v[RB][KB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int ty = t0 + rb * kWaves;
                if (ty < rows) {
                    const TIn* rp = plane + (int64_t)clampi(y_first + s0 + ty, 0, h - 1) * ish;
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        if (cv[kb]) v[rb][kb] = rp[coff[kb]];
                }
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int ty = t0 + rb * kWaves;
                if (ty < rows) {
                    TS* trow = tile + ty * TP + k0 + lane;
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        if (cv[kb]) trow[kb * 64] = to_stage<TS, TIn>(v[rb][kb]);
                }
            }
        }
    }
}

struct FragLoc {
    int f, lb, bx, by, xa, ya, bw, bh;
};

__device__ __forceinline__ FragLoc locate(const FwdLaunch& a, int gid) {
    FragLoc L;
    int f = 0;
    while (f + 1 < a.nframes && gid >= a.blk_prefix[f + 1]) ++f;
    const FrameParams& fp = a.fr[f];
    L.f = f;
    L.lb = gid - a.blk_prefix[f];
    L.by = L.lb / fp.nbx;
    L.bx = L.lb - L.by * fp.nbx;
    const int B = fp.block;
    const int X0 = fp.origin_x + L.bx * B, Y0 = fp.origin_y + L.by * B;
    L.xa = max(X0, 0);
    L.ya = max(Y0, 0);
    L.bw = min(X0 + B, a.w) - L.xa;
    L.bh = min(Y0 + B, a.h) - L.ya;
    return L;
}

template <typename TIn, typename TOut, typename TS, typename TC, int BMAX>
__global__ __launch_bounds__(kThreads) void fov_fwd_kernel(const FwdLaunch a, const int32_t* __restrict__ radius,
                                                           const TC* __restrict__ wts,
                                                           const int32_t* __restrict__ order) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int IP = BMAX + 4;
    const int gid = order[blockIdx.x];
    const FragLoc L = locate(a, gid);
    const TIn* in = static_cast<const TIn*>(a.in.data) + (int64_t)(a.frame_base + L.f) * a.in.sn;
    TOut* out = static_cast<TOut*>(a.out.data) + (int64_t)(a.frame_base + L.f) * a.out.sn;
    const int r = radius[gid];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int kWaves = kThreads / 64;

    if (r == 0) {  // foveal fragment: copied (Appendix "Workload of the Block")
        for (int c = 0; c < a.c; ++c)
            for (int y = wave; y < L.bh; y += kWaves)
                for (int x = lane; x < L.bw; x += 64) {
                    const TIn v = in[c * a.in.sc + (int64_t)(L.ya + y) * a.in.sh + (int64_t)(L.xa + x) * a.in.sw];
                    out[c * a.out.sc + (int64_t)(L.ya + y) * a.out.sh + (int64_t)(L.xa + x) * a.out.sw] =
                        copy_out<TOut, TIn>(v);
                }
        return;
    }

    const TC* __restrict__ w = wts + (size_t)gid * a.wstride;
    const Geom g = geom(r, L.bw, L.bh);
    const int SR = min(a.strip_rows, g.TH);
    const int TP = tile_pitch(g.TW, sizeof(TS));
    TS* tile = reinterpret_cast<TS*>(smem);
    TC* inter = reinterpret_cast<TC*>(smem + align16((size_t)SR * TP * sizeof(TS)));

    for (int c = 0; c < a.c; ++c) {
        const TIn* plane = in + c * a.in.sc;
        for (int s0 = 0; s0 < g.TH; s0 += SR) {
            const int rows = min(SR, g.TH - s0);
            if (s0 > 0) __syncthreads();  // every thread is done reading the previous strip
            stage_rows<TIn, TS>(tile, TP, plane, a.in.sh, a.in.sw, L.ya - r, L.xa - r, s0, rows, g.TW, a.h, a.w);
            __syncthreads();
            // Task t: lanes of a 16-lane group take 16 consecutive rows of one
            // column group, so 16-byte row reads from LDS are conflict-free.
            const int ntask = round_up(rows, 16) * g.G;
            for (int t = tid; t < ntask; t += kThreads) {
                const int blk = t >> 4, gi = blk % g.G;
                const int ty = ((blk / g.G) << 4) | (t & 15), x0 = gi * kPH;
                if (ty >= rows) continue;
                TC acc[kPH];
#pragma unroll
                for (int p = 0; p < kPH; ++p) acc[p] = 0;
                hconv(acc, tile + ty * TP + x0, g.NP, w);
                TC* dst = inter + (s0 + ty) * IP + x0;
#pragma unroll
                for (int p = 0; p < kPH; ++p) dst[p] = acc[p];
            }
        }
        __syncthreads();
        TOut* oc = out + c * a.out.sc;
        for (int t = tid; t < L.bw * g.GV; t += kThreads) {
            const int gv = t / L.bw, x = t - gv * L.bw, y0 = gv * kPV;
            TC acc[kPV];
#pragma unroll
            for (int p = 0; p < kPV; ++p) acc[p] = 0;
            vconv<IP>(acc, inter + y0 * IP + x, g.NP, w);
            TOut* o = oc + (int64_t)(L.xa + x) * a.out.sw;
#pragma unroll
            for (int p = 0; p < kPV; ++p)
                if (y0 + p < L.bh) o[(int64_t)(L.ya + y0 + p) * a.out.sh] = to_out<TOut, TC>(acc[p]);
        }
    }
}

// Fragment plan: radius and normalised taps, one wavefront per fragment.
template <typename TC>
__global__ __launch_bounds__(64) void fov_plan_weights_kernel(const FwdLaunch a, int32_t* __restrict__ radius,
                                                              TC* __restrict__ wts) {
    const int gid = blockIdx.x;
    const FragLoc L = locate(a, gid);
    const FrameParams& fp = a.fr[L.f];
    const double sigma = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[L.lb], fp.cap)
                                      : fragment_sigma_ramp(fp, L.bx, L.by);
    int r = radius_of(sigma);
    if (r > a.r_cap) r = a.r_cap;  // the host sized everything for r_cap; plans agree bit for bit
    const int lane = threadIdx.x;
    if (lane == 0) radius[gid] = r;
    const int N = 2 * r + 1;
    const double inv = r > 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
    double part = 0.0;
    for (int j = lane; j < N; j += 64) {
        const double k = (double)(j - r);
        part += exp(-(k * k) * inv);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    TC* wr = wts + (size_t)gid * a.wstride;
    for (int j = lane; j < a.wstride; j += 64) {
        double v = 0.0;
        if (j < N) {
            const double k = (double)(j - r);
            v = exp(-(k * k) * inv) / part;
        }
        wr[j] = (TC)v;
    }
}

// Dispatch order: fragments by decreasing radius (their cost grows with r),
// so the costliest start first and the launch does not end on a long tail.
// One workgroup: LDS histogram of radii, exclusive scan from the top, scatter.
// The order among equal radii is arbitrary; results do not depend on it.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 1024;

__global__ __launch_bounds__(kOrderThreads) void fov_order_kernel(const int32_t* __restrict__ radius, int n,
                                                                  int32_t* __restrict__ order) {
    __shared__ int bins[kOrderBins];
    for (int i = threadIdx.x; i < kOrderBins; i += kOrderThreads) bins[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kOrderThreads) atomicAdd(&bins[min(radius[i], kOrderBins - 1)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int b = kOrderBins - 1; b >= 0; --b) {
            const int cnt = bins[b];
            bins[b] = run;
            run += cnt;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kOrderThreads) {
        const int pos = atomicAdd(&bins[min(radius[i], kOrderBins - 1)], 1);
        order[pos] = i;
    }
}

// Device plan for foveate_plan(): sigma and radius only.
__global__ void fov_plan_kernel(FrameParams fp, int n, double* sigma_out, int32_t* r_out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int by = b / fp.nbx, bx = b - by * fp.nbx;
    double s = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[b], fp.cap) : fragment_sigma_ramp(fp, bx, by);
    if (sigma_out) sigma_out[b] = s;
    r_out[b] = radius_of(s);
}

template <typename TIn, typename TOut, typename TS, typename TC, int BMAX>
struct FwdSlot {
    static bool configured;
};
template <typename TIn, typename TOut, typename TS, typename TC, int BMAX>
bool FwdSlot<TIn, TOut, TS, TC, BMAX>::configured = false;

template <typename TIn, typename TOut, typename TS, typename TC>
fov_status launch_typed(const FwdLaunch& a, int nblocks, size_t lds, const PlanBuffers& plan, hipStream_t stream,
                        size_t lds_limit, int bmax) {
    TC* wts = static_cast<TC*>(plan.weights);
    hipLaunchKernelGGL(fov_plan_weights_kernel<TC>, dim3(nblocks), dim3(64), 0, stream, a, plan.radius, wts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "plan kernel launch");
    hipLaunchKernelGGL(fov_order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, (const int32_t*)plan.radius,
                       nblocks, plan.order);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "order kernel launch");
    auto run = [&](auto kern, bool& configured) -> fov_status {
        if (!configured) {
            hipError_t e2 = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)lds_limit);
            if (e2 != hipSuccess) return hip_error(e2, "hipFuncSetAttribute(forward)");
            configured = true;
        }
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kThreads), lds, stream, a, (const int32_t*)plan.radius,
                           (const TC*)wts, (const int32_t*)plan.order);
        hipError_t e3 = hipGetLastError();
        if (e3 != hipSuccess) return hip_error(e3, "forward kernel launch");
        return FOV_OK;
    };
    if (bmax <= 32)
        return run(fov_fwd_kernel<TIn, TOut, TS, TC, 32>, FwdSlot<TIn, TOut, TS, TC, 32>::configured);
    return run(fov_fwd_kernel<TIn, TOut, TS, TC, 64>, FwdSlot<TIn, TOut, TS, TC, 64>::configured);
}

int stage_size(int in_dtype) { return in_dtype == FOV_U8 ? 2 : (in_dtype == FOV_F32 ? 4 : 8); }
int compute_size(int in_dtype) { return in_dtype == FOV_F64 ? 8 : 4; }

}  // namespace

size_t plan_bytes(int nfrag, int wstride, int wsize) {
    return 2 * align16((size_t)nfrag * 4) + (size_t)nfrag * wstride * wsize;
}

PlanBuffers carve_plan(void* ws, int nfrag) {
    PlanBuffers p;
    char* base = static_cast<char*>(ws);
    p.radius = reinterpret_cast<int32_t*>(base);
    p.order = reinterpret_cast<int32_t*>(base + align16((size_t)nfrag * 4));
    p.weights = base + 2 * align16((size_t)nfrag * 4);
    return p;
}

size_t forward_lds_bytes(int in_dtype, int r_cap, int B, int strip_rows) {
    const int bmax = B <= 32 ? 32 : 64;
    const Geom g = geom(r_cap, B, B);
    const int rows = strip_rows < g.TH ? strip_rows : g.TH;
    const int es = stage_size(in_dtype), ec = compute_size(in_dtype);
    return align16((size_t)rows * tile_pitch(g.TW, es) * es) + (size_t)g.TH * inter_pitch(bmax) * ec + 64;
}

fov_status launch_forward(const FwdLaunch& a, int nblocks, int in_dtype, int out_dtype, size_t lds,
                          const PlanBuffers& plan, hipStream_t stream, size_t lds_limit) {
    if (nblocks <= 0) return FOV_OK;
    int bmax = 1;
    for (int i = 0; i < a.nframes; ++i) bmax = std::max(bmax, a.fr[i].block);
    if (in_dtype == FOV_U8 && out_dtype == FOV_U8)
        return launch_typed<uint8_t, uint8_t, _Float16, float>(a, nblocks, lds, plan, stream, lds_limit, bmax);
    if (in_dtype == FOV_U8 && out_dtype == FOV_F32)
        return launch_typed<uint8_t, float, _Float16, float>(a, nblocks, lds, plan, stream, lds_limit, bmax);
    if (in_dtype == FOV_F32 && out_dtype == FOV_F32)
        return launch_typed<float, float, float, float>(a, nblocks, lds, plan, stream, lds_limit, bmax);
    if (in_dtype == FOV_F64 && out_dtype == FOV_F64)
        return launch_typed<double, double, double, double>(a, nblocks, lds, plan, stream, lds_limit, bmax);
    return set_error(FOV_EDTYPE, "unsupported dtype pair");
}

fov_status launch_plan(const FrameParams& fp, int nblk, double* sigma_out, int32_t* r_out, hipStream_t stream) {
    if (nblk <= 0) return FOV_OK;
    hipLaunchKernelGGL(fov_plan_kernel, dim3((nblk + 255) / 256), dim3(256), 0, stream, fp, nblk, sigma_out, r_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "plan kernel launch");
    return FOV_OK;
}

}  // namespace fov
