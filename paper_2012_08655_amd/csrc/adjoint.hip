// Adjoint of block-wise foveation (the backward pass for training through the
// foveation), as a gather: no atomics, each output element written once.
//
// The forward map restricted to one fragment b is separable with clamp-folded
// 1-D weights: along an axis of length L, output p reads input q with weight
//     a_b(p, q) = sum over taps i in [-r_b, r_b] with clamp(p + i, 0, L-1) = q
//                 of w_b(i)
// (interior q: w_b(q - p); q = 0 collects every tap at or below the edge;
// q = L-1 every tap at or above it).  Hence
//     grad_in(qy, qx) = sum_b sum_{p in b} a_b(py, qy) a_b(px, qx) grad_out(py, px).
// A workgroup owns one tile of grad_in (aligned with the fragment grid) and
// visits every fragment whose reach [p_lo - r_b, p_hi + r_b] overlaps it;
// per fragment it forms the two small folded-weight matrices in LDS and
// applies them as a horizontal then a vertical contraction.
#include "adjoint.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>


namespace fov {

namespace {

__device__ double block_sum_d(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Folded weight a(p, q) on an axis of length L; cdf[k] = sum_{m<=k} wtab[m],
// tap index m = i + r.
__device__ __forceinline__ double folded(int p, int q, int r, int L, const double* wtab, const double* cdf) {
    if (L == 1) return cdf[2 * r];
    if (q > 0 && q < L - 1) {
        const int d = q - p;
        return (d >= -r && d <= r) ? wtab[d + r] : 0.0;
    }
    if (q == 0) {
        const int hi = -p;  // taps i <= -p land on the edge
        if (hi < -r) return 0.0;
        return cdf[min(hi, r) + r];
    }
    const int lo = max(L - 1 - p, -r);  // q == L-1: taps i >= L-1-p
    if (lo > r) return 0.0;
    return cdf[2 * r] - (lo - 1 + r >= 0 ? cdf[lo - 1 + r] : 0.0);
}

constexpr int kMaxOut = (kMaxBlock * kMaxBlock + kThreads - 1) / kThreads;

template <typename T>
__global__ __launch_bounds__(kThreads) void fov_adj_kernel(const AdjLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int gid = blockIdx.x;
    int f = 0;
    while (f + 1 < a.nframes && gid >= a.blk_prefix[f + 1]) ++f;
    const FrameParams& fp = a.fr[f];
    const int B = fp.block;
    const int nbx = fp.nbx, nby = grid_extent(a.h, fp.origin_y, B);
    const int lq = gid - a.blk_prefix[f];
    const int byq = lq / nbx, bxq = lq - byq * nbx;
    const int qx0 = max(fp.origin_x + bxq * B, 0), qy0 = max(fp.origin_y + byq * B, 0);
    const int qw = min(fp.origin_x + (bxq + 1) * B, a.w) - qx0;
    const int qh = min(fp.origin_y + (byq + 1) * B, a.h) - qy0;

    const T* g = static_cast<const T*>(a.in.data) + (int64_t)(a.frame_base + f) * a.in.sn;
    T* gi = static_cast<T*>(a.out.data) + (int64_t)(a.frame_base + f) * a.out.sn;

    T* Ax = reinterpret_cast<T*>(smem);   // [px][qx]
    T* Ay = Ax + B * B;                   // [py][qy]
    T* gb = Ay + B * B;                   // [py][px]
    T* tt = gb + B * B;                   // [py][qx]
    double* wtab = reinterpret_cast<double*>(tt + B * B);
    double* cdf = wtab + (2 * a.r_cap + 1);
    double* red = cdf + (2 * a.r_cap + 1);

    const int tid = threadIdx.x;
    const int K = (a.r_cap + B - 1) / B;
    const int nout = qw * qh;

    for (int c = 0; c < a.c; ++c) {
        T acc[kMaxOut];
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k) acc[k] = 0;
        for (int by = max(byq - K, 0); by <= min(byq + K, nby - 1); ++by)
            for (int bx = max(bxq - K, 0); bx <= min(bxq + K, nbx - 1); ++bx) {
                const int lb = by * nbx + bx;
                const double sigma = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[lb], fp.cap)
                                                  : fragment_sigma_ramp(fp, bx, by);
                int r = radius_of(sigma);
                if (r > a.r_cap) r = a.r_cap;
                const int px0 = max(fp.origin_x + bx * B, 0), py0 = max(fp.origin_y + by * B, 0);
                const int bw = min(fp.origin_x + (bx + 1) * B, a.w) - px0;
                const int bh = min(fp.origin_y + (by + 1) * B, a.h) - py0;
                // reach along each axis (clamping keeps edge taps inside the frame)
                if (px0 - r > qx0 + qw - 1 || px0 + bw - 1 + r < qx0) continue;
                if (py0 - r > qy0 + qh - 1 || py0 + bh - 1 + r < qy0) continue;
                const int N = 2 * r + 1;
                // weights of fragment b, normalised, and their running sum
                double part = 0.0;
                const double inv = r > 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
                for (int j = tid; j < N; j += kThreads) {
                    const double k = (double)(j - r);
                    const double v = r > 0 ? exp(-(k * k) * inv) : 1.0;
                    wtab[j] = v;
                    part += v;
                }
                const double S = block_sum_d(part, red);  // syncs: wtab complete
                for (int j = tid; j < N; j += kThreads) wtab[j] /= S;
                __syncthreads();
                if (tid == 0) {
                    double s = 0.0;
                    for (int j = 0; j < N; ++j) { s += wtab[j]; cdf[j] = s; }
                }
                __syncthreads();
                for (int i = tid; i < bw * qw; i += kThreads) {
                    const int p = i / qw, q = i - p * qw;
                    Ax[p * B + q] = (T)folded(px0 + p, qx0 + q, r, a.w, wtab, cdf);
                }
                for (int i = tid; i < bh * qh; i += kThreads) {
                    const int p = i / qh, q = i - p * qh;
                    Ay[p * B + q] = (T)folded(py0 + p, qy0 + q, r, a.h, wtab, cdf);
                }
                for (int i = tid; i < bh * bw; i += kThreads) {
                    const int y = i / bw, x = i - y * bw;
                    gb[y * B + x] = g[c * a.in.sc + (int64_t)(py0 + y) * a.in.sh + (int64_t)(px0 + x) * a.in.sw];
                }
                __syncthreads();
                // horizontal contraction: tt[py][qx] = sum_px gb[py][px] * Ax[px][qx]
                for (int i = tid; i < bh * qw; i += kThreads) {
                    const int y = i / qw, q = i - y * qw;
                    T s = 0;
                    for (int x = 0; x < bw; ++x) s = fma(gb[y * B + x], Ax[x * B + q], s);
                    tt[y * B + q] = s;
                }
                __syncthreads();
                // vertical contraction into this thread's outputs
#pragma unroll
                for (int k = 0; k < kMaxOut; ++k) {
                    const int i = tid + k * kThreads;
                    if (i < nout) {
                        const int qy = i / qw, qx = i - qy * qw;
                        T s = acc[k];
                        for (int y = 0; y < bh; ++y) s = fma(Ay[y * B + qy], tt[y * B + qx], s);
                        acc[k] = s;
                    }
                }
                __syncthreads();
            }
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k) {
            const int i = tid + k * kThreads;
            if (i < nout) {
                const int qy = i / qw, qx = i - qy * qw;
                gi[c * a.out.sc + (int64_t)(qy0 + qy) * a.out.sh + (int64_t)(qx0 + qx) * a.out.sw] = acc[k];
            }
        }
    }
}

template <typename T>
struct AdjSlot {
    static bool configured;
};
template <typename T>
bool AdjSlot<T>::configured = false;

template <typename T>
fov_status launch_adj_typed(const AdjLaunch& a, int nblocks, size_t lds, hipStream_t stream, size_t lds_limit) {
    auto kern = fov_adj_kernel<T>;
    if (!AdjSlot<T>::configured) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit);
        if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(adjoint)");
        AdjSlot<T>::configured = true;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kThreads), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint kernel launch");
    return FOV_OK;
}

}  // namespace

size_t adjoint_lds_bytes(int r_cap, int B, int es) {
    return (size_t)4 * B * B * es + (size_t)2 * (2 * r_cap + 1) * 8 + 64;
}

fov_status launch_adjoint_all(const fov_tensor* go, const fov_tensor* gi, const fov_params* p, int32_t np,
                              hipStream_t stream, size_t lds_limit) {
    const int es = go->dtype == FOV_F64 ? 8 : 4;
    for (int f0 = 0; f0 < go->n; f0 += kMaxFramesPerLaunch) {
        const int nf = std::min(kMaxFramesPerLaunch, go->n - f0);
        AdjLaunch a;
        std::memset(&a, 0, sizeof(a));
        a.in = View{go->data, go->sn, go->sc, go->sh, go->sw};
        a.out = View{gi->data, gi->sn, gi->sc, gi->sh, gi->sw};
        a.c = go->c; a.h = go->h; a.w = go->w;
        a.nframes = nf;
        a.frame_base = f0;
        int r_cap = 0, bmax = 1, total = 0;
        for (int i = 0; i < nf; ++i) {
            const fov_params& pp = p[np == 1 ? 0 : f0 + i];
            FrameParams& fr = a.fr[i];
            fr.fix_x = pp.fix_x; fr.fix_y = pp.fix_y; fr.e0 = pp.e0; fr.slope = pp.slope; fr.cap = pp.cap;
            fr.block = pp.block; fr.origin_x = pp.origin_x; fr.origin_y = pp.origin_y;
            fr.nbx = grid_extent(go->w, pp.origin_x, pp.block);
            fr.sigma_map = pp.sigma_map;
            a.blk_prefix[i] = total;
            const int nby = grid_extent(go->h, pp.origin_y, pp.block);
            total += fr.nbx * nby;
            int rm = 0;
            if (pp.sigma_map) {
                rm = radius_of(pp.cap);
            } else {
                const int xs[2] = {0, fr.nbx - 1}, ys[2] = {0, nby - 1};
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) rm = std::max(rm, radius_of(fragment_sigma_ramp(fr, xs[u], ys[v])));
            }
            r_cap = std::max(r_cap, rm);
            bmax = std::max(bmax, pp.block);
        }
        a.blk_prefix[nf] = total;
        a.r_cap = r_cap;
        const size_t lds = adjoint_lds_bytes(r_cap, bmax, es);
        if (lds > lds_limit) return set_error(FOV_ERANGE, "adjoint tile does not fit in LDS");
        fov_status s = es == 8 ? launch_adj_typed<double>(a, total, lds, stream, lds_limit)
                               : launch_adj_typed<float>(a, total, lds, stream, lds_limit);
        if (s != FOV_OK) return s;
    }
    return FOV_OK;
}

}  // namespace fov
