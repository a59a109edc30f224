// Forward block-wise foveation kernel for gfx950.
//
// One workgroup per output fragment (Sec. 2, Alg. 1): the fragment's sigma
// and radius come from its midpoint's eccentricity; the padded tile is staged
// into LDS with coalesced row reads and clamp-to-edge indexing; a horizontal
// pass writes an fp32 intermediate into LDS; a vertical pass over that
// intermediate produces the output fragment (Appendix "Workload of the
// Block", "Shared Memory").  Each thread computes several outputs and slides
// the filter window through registers so every staged value is read from LDS
// once per thread (the data-reuse scheme of Appendix "Data Reuse").
//
// Weights w_k = exp(-k^2 / (2 sigma^2)) are built per workgroup in double,
// summed with a wavefront-shuffle reduction, normalised and stored in LDS
// zero-padded to a multiple of 8 taps; every output sums its taps in the same
// order (k = -r .. r), independent of tiling choices.
#include "forward.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace fov {

namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec4<double> { using type = double2; static constexpr int n = 2; };

template <typename TIn, typename TC>
__device__ __forceinline__ TC to_compute(TIn v) { return (TC)v; }

template <typename TOut, typename TC>
__device__ __forceinline__ TOut from_compute(TC v) { return (TOut)v; }
template <>
__device__ __forceinline__ uint8_t from_compute<uint8_t, float>(float v) {
    v = rintf(v);  // round half to even
    v = fminf(fmaxf(v, 0.0f), 255.0f);
    return (uint8_t)v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Sum over the workgroup with wavefront shuffles, then across waves in LDS.
__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Load U contiguous LDS elements at p (16-byte aligned) into buf.
template <int U, typename T>
__device__ __forceinline__ void lds_load_row(const T* p, T (&buf)[U]) {
    using V = typename Vec4<T>::type;
    constexpr int n = Vec4<T>::n;
#pragma unroll
    for (int k = 0; k < U; k += n) {
        V v = *reinterpret_cast<const V*>(p + k);
        if constexpr (n == 4) {
            buf[k] = v.x; buf[k + 1] = v.y; buf[k + 2] = v.z; buf[k + 3] = v.w;
        } else {
            buf[k] = v.x; buf[k + 1] = v.y;
        }
    }
}

// Load U LDS elements spaced by `pitch` starting at p.
template <int U, typename T>
__device__ __forceinline__ void lds_load_col(const T* p, int pitch, T (&buf)[U]) {
#pragma unroll
    for (int k = 0; k < U; ++k) buf[k] = p[k * pitch];
}

// One window step: taps j0..j0+U-1 applied to P outputs whose inputs are the
// concatenation A ++ B (A holds inputs j0..j0+U-1 relative to output 0).
template <int P, int U, typename T>
__device__ __forceinline__ void window_step(T (&acc)[P], const T (&A)[U], const T (&B)[U], const T* w) {
    static_assert(P <= U + 1, "window must fit in two buffers");
    T wr[U];
    lds_load_row<U>(w, wr);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i = p + u;
            const T v = i < U ? A[i] : B[i - U];
            acc[p] = fma(wr[u], v, acc[p]);
        }
}

// P outputs of a 1-D convolution with NP (multiple of U) taps; `load(i, buf)`
// fills buf with inputs i..i+U-1 relative to the first output.  Reads inputs
// up to NP+U-1.
template <int P, int U, typename T, typename Load>
__device__ __forceinline__ void conv_slide(T (&acc)[P], int NP, const T* wts, Load load) {
    T A[U], B[U];
    load(0, A);
    int j0 = 0;
    for (; j0 + 2 * U <= NP; j0 += 2 * U) {
        load(j0 + U, B);
        window_step<P, U>(acc, A, B, wts + j0);
        load(j0 + 2 * U, A);
        window_step<P, U>(acc, B, A, wts + j0 + U);
    }
    if (j0 < NP) {
        load(j0 + U, B);
        window_step<P, U>(acc, A, B, wts + j0);
    }
}

template <typename TIn, typename TOut, typename TC>
__global__ __launch_bounds__(kThreads) void fov_fwd_kernel(const FwdLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];

    // ---- locate fragment ------------------------------------------------------
    const int gid = blockIdx.x;
    int f = 0;
    while (f + 1 < a.nframes && gid >= a.blk_prefix[f + 1]) ++f;
    const FrameParams& fp = a.fr[f];
    const int lb = gid - a.blk_prefix[f];
    const int by = lb / fp.nbx, bx = lb - by * fp.nbx;
    const int B = fp.block;
    const int X0 = fp.origin_x + bx * B, Y0 = fp.origin_y + by * B;
    const int xa = max(X0, 0), ya = max(Y0, 0);
    const int bw = min(X0 + B, a.w) - xa, bh = min(Y0 + B, a.h) - ya;

    const TIn* in = static_cast<const TIn*>(a.in.data) + (int64_t)(a.frame_base + f) * a.in.sn;
    TOut* out = static_cast<TOut*>(a.out.data) + (int64_t)(a.frame_base + f) * a.out.sn;

    // ---- plan: sigma and radius of this fragment --------------------------------
    double sigma = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[lb], fp.cap)
                                : fragment_sigma_ramp(fp, bx, by);
    int r = radius_of(sigma);
    if (r > a.r_cap) r = a.r_cap;  // host sized LDS for r_cap; never taken when plans agree

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    constexpr int kWaves = kThreads / 64;

    if (r == 0) {  // foveal fragment: copy (Appendix "Workload of the Block")
        for (int c = 0; c < a.c; ++c)
            for (int y = wave; y < bh; y += kWaves)
                for (int x = lane; x < bw; x += 64) {
                    TIn v = in[c * a.in.sc + (int64_t)(ya + y) * a.in.sh + (int64_t)(xa + x) * a.in.sw];
                    out[c * a.out.sc + (int64_t)(ya + y) * a.out.sh + (int64_t)(xa + x) * a.out.sw] =
                        from_compute<TOut, TC>(to_compute<TIn, TC>(v));
                }
        return;
    }

    const TileGeom g = tile_geom(r, bw, bh);
    const int N = 2 * r + 1;
    TC* wts = reinterpret_cast<TC*>(smem);
    TC* strip = wts + round_up(g.NP, 4);
    const int SR = min(a.strip_rows, g.TH);
    TC* inter = strip + (size_t)SR * g.TP;
    double* red = reinterpret_cast<double*>(inter + (size_t)g.TH * g.IP);

    // ---- weights: Eq. (1) sampled at integer offsets, cut at r, normalised ------
    {
        double wv = 0.0;
        const double inv = 1.0 / (2.0 * sigma * sigma);
        for (int j = tid; j < N; j += kThreads) {
            const double k = (double)(j - r);
            wv += exp(-(k * k) * inv);
        }
        const double S = block_sum(wv, red);
        for (int j = tid; j < g.NP; j += kThreads) {
            double v = 0.0;
            if (j < N) {
                const double k = (double)(j - r);
                v = exp(-(k * k) * inv) / S;
            }
            wts[j] = (TC)v;
        }
    }

    const int G = (bw + kPH - 1) / kPH;          // horizontal-pass column groups
    const int GV = (bh + kPV - 1) / kPV;         // vertical-pass row groups
    const int64_t isc = a.in.sc, ish = a.in.sh, isw = a.in.sw;

    for (int c = 0; c < a.c; ++c) {
        const TIn* inc = in + c * isc;
        // ---- horizontal pass, streamed through LDS in strips of SR tile rows ----
        for (int s0 = 0; s0 < g.TH; s0 += SR) {
            const int rows = min(SR, g.TH - s0);
            __syncthreads();  // previous strip / weights / previous channel done
            for (int ty = wave; ty < rows; ty += kWaves) {
                const int gy = clampi(ya - r + s0 + ty, 0, a.h - 1);
                const TIn* src = inc + (int64_t)gy * ish;
                TC* dst = strip + ty * g.TP;
                for (int tx = lane; tx < g.TW; tx += 64) {
                    const int gx = clampi(xa - r + tx, 0, a.w - 1);
                    dst[tx] = to_compute<TIn, TC>(src[(int64_t)gx * isw]);
                }
            }
            __syncthreads();
            for (int t = tid; t < rows * G; t += kThreads) {
                const int ty = t / G, x0 = (t - ty * G) * kPH;
                TC acc[kPH];
#pragma unroll
                for (int p = 0; p < kPH; ++p) acc[p] = 0;
                const TC* row = strip + ty * g.TP + x0;
                conv_slide<kPH, kU>(acc, g.NP, wts, [&](int i, TC (&buf)[kU]) { lds_load_row<kU>(row + i, buf); });
                TC* dst = inter + (s0 + ty) * g.IP + x0;
#pragma unroll
                for (int p = 0; p < kPH; ++p) dst[p] = acc[p];
            }
        }
        __syncthreads();
        // ---- vertical pass over the intermediate, write the fragment ------------
        for (int t = tid; t < bw * GV; t += kThreads) {
            const int gy = t / bw, x = t - gy * bw, y0 = gy * kPV;
            TC acc[kPV];
#pragma unroll
            for (int p = 0; p < kPV; ++p) acc[p] = 0;
            const TC* col = inter + y0 * g.IP + x;
            const int ip = g.IP;
            conv_slide<kPV, kU>(acc, g.NP, wts, [&](int i, TC (&buf)[kU]) { lds_load_col<kU>(col + i * ip, ip, buf); });
            TOut* o = out + c * a.out.sc + (int64_t)(xa + x) * a.out.sw;
#pragma unroll
            for (int p = 0; p < kPV; ++p)
                if (y0 + p < bh) o[(int64_t)(ya + y0 + p) * a.out.sh] = from_compute<TOut, TC>(acc[p]);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Device plan: the same sigma/radius code the kernel runs, written to memory.
__global__ void fov_plan_kernel(FrameParams fp, int n, double* sigma_out, int32_t* r_out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int by = b / fp.nbx, bx = b - by * fp.nbx;
    double s = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[b], fp.cap) : fragment_sigma_ramp(fp, bx, by);
    if (sigma_out) sigma_out[b] = s;
    r_out[b] = radius_of(s);
}

template <typename TIn, typename TOut, typename TC>
struct KernelSlot {
    static bool configured;
};
template <typename TIn, typename TOut, typename TC>
bool KernelSlot<TIn, TOut, TC>::configured = false;

template <typename TIn, typename TOut, typename TC>
fov_status launch_typed(const FwdLaunch& a, int nblocks, size_t lds, hipStream_t stream, size_t lds_limit) {
    auto kern = fov_fwd_kernel<TIn, TOut, TC>;
    if (!KernelSlot<TIn, TOut, TC>::configured) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit);
        if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(forward)");
        KernelSlot<TIn, TOut, TC>::configured = true;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kThreads), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "forward kernel launch");
    return FOV_OK;
}

}  // namespace

fov_status launch_forward(const FwdLaunch& a, int nblocks, int in_dtype, int out_dtype, size_t lds,
                          hipStream_t stream, size_t lds_limit) {
    if (nblocks <= 0) return FOV_OK;
    if (in_dtype == FOV_U8 && out_dtype == FOV_U8)
        return launch_typed<uint8_t, uint8_t, float>(a, nblocks, lds, stream, lds_limit);
    if (in_dtype == FOV_U8 && out_dtype == FOV_F32)
        return launch_typed<uint8_t, float, float>(a, nblocks, lds, stream, lds_limit);
    if (in_dtype == FOV_F32 && out_dtype == FOV_F32)
        return launch_typed<float, float, float>(a, nblocks, lds, stream, lds_limit);
    if (in_dtype == FOV_F64 && out_dtype == FOV_F64)
        return launch_typed<double, double, double>(a, nblocks, lds, stream, lds_limit);
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
