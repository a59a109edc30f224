// Adjoint of block-wise foveation (the backward pass for training through the
// foveation), as a gather: no atomics, every element written once, a fixed
// summation order.
//
// Restricted to one fragment b, the forward map is separable: a horizontal
// then a vertical 1-D correlation with b's taps w_b over the clamped frame.
// Its transpose maps the fragment's output gradient g_b back over b's
// padded window, so
//     grad_in = sum_b Fold_y V_b^T Fold_x H_b^T g_b,
// where H_b^T / V_b^T correlate with w_b (the taps are symmetric) over the
// fragment's rows / columns padded by r_b, and Fold adds what lands outside
// the frame onto the edge row or column (the transpose of clamp-to-edge).
// On an axis of length L the fold gives output 0 the extra weight
// cdf_b(-p-1) = sum_{i <= -p-1} w_b(i) for input p, and output L-1 the extra
// weight cdf_b(p-L).
//
// Two kernels after the plan kernel (radius and taps of every fragment):
//  1. fov_adj_h_kernel — one workgroup per fragment: the horizontal transpose
//     Fold_x H_b^T g_b (rows of b, columns of b's reach) into a scratch buffer.
//     Lanes take rows; a wave shares one group of 8 output columns, so the
//     taps that meet the fragment form one wave-uniform range.
//  2. fov_adj_v_kernel — one workgroup per output tile (the fragment grid):
//     for every fragment b whose reach meets the tile, stage b's scratch rows
//     over the tile's columns (zero-padded, several channels at once) in LDS
//     and accumulate the vertical transpose in registers; the fragments are
//     visited in a fixed order.
// Both passes are the forward's register-window correlations with the taps
// read as scalar operands, run over the band of taps that meet the fragment.
#include "adjoint.h"

#include <hip/hip_runtime.h>

#include <algorithm>

#include "conv.h"

namespace fov {

namespace {

constexpr int kPadA = 12;  // zero columns staged before a fragment row (horizontal kernel)

__global__ void fov_adj_lead_kernel(unsigned char* p, int bytes) {
    for (int i = threadIdx.x; i < bytes; i += blockDim.x) p[i] = 0;
}

// Horizontal transpose of fragment gid into scratch[gid][c][row][x - xa + r_cap]
// for the columns x of its clamped reach.
template <typename T>
__global__ __launch_bounds__(kThreads) void fov_adj_h_kernel(const FwdLaunch a, const AdjShape s,
                                                             const FrameDesc* __restrict__ table,
                                                             const int32_t* __restrict__ prefix,
                                                             const int32_t* __restrict__ radius,
                                                             const T* __restrict__ wts, T* __restrict__ scratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* rows = reinterpret_cast<T*>(smem);  // [chunk_c * bh][pitch_a]
    constexpr int V = 16 / sizeof(T);      // elements per aligned 16-byte LDS load
    const int gid = blockIdx.x;
    const Frag F = describe(table, prefix, a.nframes, gid);
    const FrameDesc& d = *F.fd;
    const int r = radius[gid];
    const T* __restrict__ w = wts + (size_t)gid * a.wstride;
    const int xs = max(F.xa - r, 0), xe = min(F.xa + F.bw - 1 + r, d.w - 1);
    const int G = (xe - xs + kPH) / kPH;
    const T* g = static_cast<const T*>(d.in);
    const int P = s.pitch_a;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    for (int c0 = 0; c0 < d.c; c0 += s.chunk_c) {
        const int cc = min(s.chunk_c, d.c - c0);
        const int RT = cc * F.bh;
        if (c0 > 0) __syncthreads();  // previous channels' rows are no longer read
        for (int row = wave; row < RT; row += kThreads / 64) {  // a wave per row, lanes along it
            const int k = row / F.bh, py = row - k * F.bh;
            const T* grow = g + (int64_t)(c0 + k) * d.isc + (int64_t)(F.ya + py) * d.ish + (int64_t)F.xa * d.isw;
            T* lrow = rows + row * P;
            for (int col = lane; col < P; col += 64) {
                const int x = col - kPadA;
                lrow[col] = (x >= 0 && x < F.bw) ? grow[(int64_t)x * d.isw] : (T)0;
            }
        }
        __syncthreads();
        const int nchunk = (RT + 63) / 64;
        for (int task = wave; task < nchunk * G; task += kThreads / 64) {
            const int gi = task / nchunk, ch = task - gi * nchunk;
            const int X = xs + gi * kPH;
            // taps t with X + p + t inside the fragment for some p in 0..7
            int t_lo = max(-r, F.xa - X - (kPH - 1));
            const int t_hi = min(r, F.xa + F.bw - 1 - X);
            const int row = ch * 64 + lane;
            if (row >= RT) continue;
            const T* rr = rows + row * P + kPadA - F.xa;  // rr[x]: this row's gradient at frame column x
            T acc[kPH];
#pragma unroll
            for (int p = 0; p < kPH; ++p) acc[p] = 0;
            if (t_lo <= t_hi) {
                t_lo -= (X + t_lo - F.xa + kPadA) & (V - 1);  // aligned window start; taps below -r are zero
                hconv(acc, rr + X + t_lo, t_hi - t_lo + 1, w + (t_lo + r));
            }
            if (xs == 0 && gi == 0) {  // column 0 collects the taps that fell off the left edge
                T cdf = 0, corr = 0;
                for (int m = -r; m <= -F.xa - 1; ++m) {
                    cdf += w[m + r];
                    const int x = -m - 1;
                    if (x < F.xa + F.bw) corr = fma(cdf, rr[x], corr);
                }
                acc[0] += corr;
            }
            const int jr = d.w - 1 - X;
            if (xe == d.w - 1 && jr >= 0 && jr < kPH) {  // column w-1 collects those off the right edge
                T cdf = 0, corr = 0;
                for (int m = -r; m <= -1; ++m) {
                    cdf += w[m + r];
                    const int x = m + d.w;
                    if (x >= F.xa && x < F.xa + F.bw) corr = fma(cdf, rr[x], corr);
                }
#pragma unroll
                for (int p = 0; p < kPH; ++p)
                    if (p == jr) acc[p] += corr;
            }
            const int k = row / F.bh, py = row - k * F.bh;
            T* dst = scratch + (((size_t)gid * s.cmax + (c0 + k)) * s.bmax + py) * s.sw + (X - F.xa + a.r_cap);
#pragma unroll
            for (int p = 0; p < kPH; ++p)
                if (X + p <= xe) dst[p] = acc[p];
        }
    }
}

// Vertical gather into output tile gid: grad_in over the tile's rectangle.
// TASKS: output tasks per thread (4 rows of one column each), CB: channels
// staged and accumulated together, so each neighbouring fragment costs one
// staging round per CB channels.
template <typename T, int TASKS, int CB>
__global__ __launch_bounds__(kThreads) void fov_adj_v_kernel(const FwdLaunch a, const AdjShape s,
                                                             const FrameDesc* __restrict__ table,
                                                             const int32_t* __restrict__ prefix,
                                                             const int32_t* __restrict__ radius,
                                                             const T* __restrict__ wts,
                                                             const T* __restrict__ scratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* cols = reinterpret_cast<T*>(smem);  // [CB channels][bmax columns][pitch_b rows]
    constexpr int V = 16 / sizeof(T);
    const int gid = blockIdx.x;
    const Frag Q = describe(table, prefix, a.nframes, gid);
    const FrameDesc& d = *Q.fd;
    const FrameParams& fp = d.p;
    const int nbx = fp.nbx, nby = d.nby;
    const int first = gid - Q.lb;
    const int K = (a.r_cap + fp.block - 1) / fp.block;  // fragments within reach on each side
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const int PB = s.pitch_b, PAD = s.pad_b;
    const int CS = s.bmax * PB;  // one staged channel
    const int ngroups = (Q.bh + kPV - 1) / kPV;
    const int ntask = s.bmax * ngroups;  // task i: column i % bmax, rows 4 (i / bmax) .. +3
    const int by_lo = max(Q.by - K, 0), by_hi = min(Q.by + K, nby - 1);
    const int bx_lo = max(Q.bx - K, 0), bx_hi = min(Q.bx + K, nbx - 1);
    T* out = static_cast<T*>(d.out);
    // The PAD rows above and the rows below bmax stay zero: staged once here, never written again
    // (each round writes rows PAD .. PAD + bmax - 1 only; the first round's barrier orders this).
    for (int i = tid; i < s.chunk_v * CS; i += kThreads) cols[i] = (T)0;  // the slots allocated (<= CB)
    const int rg_lo = PAD / V, rg_hi = (PAD + s.bmax + V - 1) / V;  // row groups that can hold b's rows
    for (int c0 = 0; c0 < d.c; c0 += CB) {
        const int cc = min(CB, d.c - c0);
        T acc[CB][TASKS][kPV];
#pragma unroll
        for (int ch = 0; ch < CB; ++ch)
#pragma unroll
            for (int k = 0; k < TASKS; ++k)
#pragma unroll
                for (int p = 0; p < kPV; ++p) acc[ch][k][p] = 0;
        for (int by = by_lo; by <= by_hi; ++by)
            for (int bx = bx_lo; bx <= bx_hi; ++bx) {
                const int b = first + by * nbx + bx;
                const Frag Fb = describe_at(Q.fd, first, b);
                const int r = radius[b];
                const int rx0 = max(Fb.xa - r, 0), rx1 = min(Fb.xa + Fb.bw - 1 + r, d.w - 1);
                const int ry0 = max(Fb.ya - r, 0), ry1 = min(Fb.ya + Fb.bh - 1 + r, d.h - 1);
                if (rx1 < Q.xa || rx0 >= Q.xa + Q.bw || ry1 < Q.ya || ry0 >= Q.ya + Q.bh) continue;
                const T* __restrict__ w = wts + (size_t)b * a.wstride;
                const int xoff = a.r_cap - Fb.xa;
                __syncthreads();  // the previous fragment's columns are no longer read
                // per channel, column x of the tile: b's rows from row PAD on (zeros past its height
                // and outside its reach)
                const int nrg = rg_hi - rg_lo;
                const int items = Q.bw * nrg;
                for (int i = tid; i < cc * items; i += kThreads) {
                    const int ch = i / items, j = i - ch * items;
                    const int rg = rg_lo + j / Q.bw, x = j - (j / Q.bw) * Q.bw;
                    const int gx = Q.xa + x;
                    const bool inx = gx >= rx0 && gx <= rx1;
                    const T* src = scratch + ((size_t)b * s.cmax + c0 + ch) * s.bmax * s.sw;
                    T v[V];
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int py = rg * V + u - PAD;
                        v[u] = (inx && py >= 0 && py < Fb.bh) ? src[(size_t)py * s.sw + gx + xoff] : (T)0;
                    }
                    T* dst = cols + ch * CS + x * PB + rg * V;
                    if constexpr (V == 4) {
                        *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
                        *reinterpret_cast<double2*>(dst) = make_double2(v[0], v[1]);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < TASKS; ++k) {
                    const int i0 = wave * 64 + k * kThreads;
                    if (i0 >= ntask) break;
                    // taps t with y + t inside fragment b for some row y of this wave
                    const int gA = i0 / s.bmax, gB = min((i0 + 63) / s.bmax, ngroups - 1);
                    const int ymin = Q.ya + kPV * gA, ymax = min(Q.ya + kPV * gB + kPV - 1, Q.ya + Q.bh - 1);
                    int t_lo = max(-r, Fb.ya - ymax);
                    const int t_hi = min(r, Fb.ya + Fb.bh - 1 - ymin);
                    if (t_lo <= t_hi) t_lo -= (Q.ya + t_lo - Fb.ya + PAD) & (V - 1);  // aligned window start
                    const int i = i0 + lane;
                    const int x = i % s.bmax, gr = i / s.bmax;
                    if (x >= Q.bw || gr >= ngroups) continue;
                    const int y0 = Q.ya + kPV * gr;
                    const bool top = y0 == 0;           // row 0 collects the taps off the top edge
                    const int pr = d.h - 1 - y0;        // row h-1 collects those off the bottom edge
                    const bool bottom = pr >= 0 && pr < kPV;
#pragma unroll
                    for (int ch = 0; ch < CB; ++ch) {
                        if (ch >= cc) break;
                        const T* col = cols + ch * CS + x * PB + PAD - Fb.ya;  // col[y]: b's transpose at row y
                        if (t_lo <= t_hi) vconv(acc[ch][k], col + y0 + t_lo, t_hi - t_lo + 1, w + (t_lo + r));
                        if (top) {
                            T cdf = 0, corr = 0;
                            for (int m = -r; m <= -Fb.ya - 1; ++m) {
                                cdf += w[m + r];
                                const int py = -m - 1;
                                if (py < Fb.ya + Fb.bh) corr = fma(cdf, col[py], corr);
                            }
                            acc[ch][k][0] += corr;
                        }
                        if (bottom) {
                            T cdf = 0, corr = 0;
                            for (int m = -r; m <= -1; ++m) {
                                cdf += w[m + r];
                                const int py = m + d.h;
                                if (py >= Fb.ya && py < Fb.ya + Fb.bh) corr = fma(cdf, col[py], corr);
                            }
#pragma unroll
                            for (int p = 0; p < kPV; ++p)
                                if (p == pr) acc[ch][k][p] += corr;
                        }
                    }
                }
            }
#pragma unroll
        for (int k = 0; k < TASKS; ++k) {
            const int i = wave * 64 + k * kThreads + lane;
            if (i >= ntask) break;
            const int x = i % s.bmax, gr = i / s.bmax;
            if (x >= Q.bw || gr >= ngroups) continue;
#pragma unroll
            for (int ch = 0; ch < CB; ++ch) {
                if (ch >= cc) break;
                T* o = out + (c0 + ch) * d.osc + (int64_t)(Q.xa + x) * d.osw;
#pragma unroll
                for (int p = 0; p < kPV; ++p) {
                    const int y = Q.ya + kPV * gr + p;
                    if (y < Q.ya + Q.bh) o[(int64_t)y * d.osh] = acc[ch][k][p];
                }
            }
        }
    }
}

template <typename T, int TASKS, int CB>
fov_status launch_typed(const FwdLaunch& a, const AdjShape& s, const PlanBuffers& plan, void* scratch,
                        hipStream_t stream, size_t lds_limit) {
    auto kh = fov_adj_h_kernel<T>;
    auto kv = fov_adj_v_kernel<T, TASKS, CB>;
    fov_status st;
    if ((st = allow_dyn_lds((const void*)kh, lds_limit)) != FOV_OK) return st;
    if ((st = allow_dyn_lds((const void*)kv, lds_limit)) != FOV_OK) return st;
    const T* wts = static_cast<const T*>(plan.weights);
    T* sc = static_cast<T*>(scratch);
    hipLaunchKernelGGL(kh, dim3(a.nfrag), dim3(kThreads), adjoint_lds_h(s, sizeof(T)), stream, a, s,
                       (const FrameDesc*)a.table, (const int32_t*)a.prefix, (const int32_t*)plan.radius, wts, sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint horizontal kernel launch");
    hipLaunchKernelGGL(kv, dim3(a.nfrag), dim3(kThreads), adjoint_lds_v(s, sizeof(T)), stream, a, s,
                       (const FrameDesc*)a.table, (const int32_t*)a.prefix, (const int32_t*)plan.radius, wts,
                       (const T*)sc);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint vertical kernel launch");
    return FOV_OK;
}

template <typename T>
fov_status launch_for_tasks(const FwdLaunch& a, const AdjShape& s, const PlanBuffers& plan, void* scratch,
                            hipStream_t stream, size_t lds_limit) {
    if (s.tasks_v == 1) return launch_typed<T, 1, 4>(a, s, plan, scratch, stream, lds_limit);
    if (s.tasks_v == 2) return launch_typed<T, 2, 2>(a, s, plan, scratch, stream, lds_limit);
    return launch_typed<T, 4, 1>(a, s, plan, scratch, stream, lds_limit);
}

}  // namespace

AdjShape adjoint_shape(int es, int r_cap, int bmax, int cmax) {
    AdjShape s;
    s.bmax = bmax;
    s.sw = bmax + 2 * r_cap;
    s.cmax = cmax;
    s.pitch_a = tile_pitch(bmax + kPadA + 7, es);
    s.chunk_c = std::max(1, std::min(cmax, 128 / bmax));
    // rows one wave's tasks span in the vertical kernel, minus one
    const int span = std::min(kPV * (63 / bmax + 1) + kPV - 1, bmax - 1);
    s.pad_b = round_up(span + 4, 4);
    s.pitch_b = inter_pitch(bmax + 2 * s.pad_b, es);
    // vertical kernel: tasks of 4 rows x 1 column per thread (1, 2 or 4) and
    // channels staged together (4 / tasks, at most the channel count)
    const int tasks = (bmax * ((bmax + kPV - 1) / kPV) + kThreads - 1) / kThreads;
    s.tasks_v = tasks <= 1 ? 1 : (tasks <= 2 ? 2 : 4);
    s.chunk_v = std::max(1, std::min(cmax, 4 / s.tasks_v));
    return s;
}

size_t adjoint_lds_h(const AdjShape& s, int es) { return (size_t)s.chunk_c * s.bmax * s.pitch_a * es; }

size_t adjoint_lds_v(const AdjShape& s, int es) { return (size_t)s.chunk_v * s.bmax * s.pitch_b * es; }

size_t adjoint_scratch_elems(const AdjShape& s, int nfrag) {
    return (size_t)nfrag * s.cmax * s.bmax * s.sw;
}

fov_status launch_adjoint(const FwdLaunch& a, const AdjShape& s, int es, const PlanBuffers& plan, void* weights_base,
                          void* scratch, hipStream_t stream, size_t lds_limit) {
    if (a.nfrag <= 0) return FOV_OK;
    if (adjoint_lds_h(s, es) + 64 > lds_limit || adjoint_lds_v(s, es) + 64 > lds_limit)
        return set_error(FOV_ERANGE, "adjoint tiles do not fit in LDS");
    hipLaunchKernelGGL(fov_adj_lead_kernel, dim3(1), dim3(64), 0, stream, static_cast<unsigned char*>(weights_base),
                       kAdjWeightLead * es);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint lead kernel launch");
    fov_status st = launch_plan_weights(a, es, plan, stream);
    if (st != FOV_OK) return st;
    return es == 8 ? launch_for_tasks<double>(a, s, plan, scratch, stream, lds_limit)
                   : launch_for_tasks<float>(a, s, plan, scratch, stream, lds_limit);
}

}  // namespace fov
