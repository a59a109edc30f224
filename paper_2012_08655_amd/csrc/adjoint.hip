// Adjoint of block-wise foveation (the backward pass for training through the
// foveation), as a gather: no atomics, every element written once, a fixed
// summation order.
//
// Restricted to one fragment b, the forward map is separable: a horizontal
// then a vertical 1-D correlation with b's taps w_b over the clamped frame.
// Its transpose maps the fragment's output gradient g_b back over b's window
// (the fragment grown by r_b on every side), so
//     grad_in = sum_b Fold_x H_b^T Fold_y V_b^T g_b,
// where V_b^T / H_b^T correlate with w_b (the taps are symmetric) over the
// window's rows / columns, and Fold adds what lands outside the frame onto
// the edge row or column (the transpose of clamp-to-edge).  On an axis of
// length L the fold gives output 0 the extra weight
// cdf_b(-p-1) = sum_{i <= -p-1} w_b(i) for input p, and output L-1 the extra
// weight cdf_b(p-L).
//
// Two kernels:
//  1. fov_adj_window_kernel — one workgroup per fragment and channel: the
//     fragment's sigma, radius and normalised taps (kept in LDS), then its
//     transposed window as the forward computes a fragment: the gradient is
//     staged in LDS (column-major, zero rows around it), the vertical
//     transpose writes the window's rows into a second LDS buffer (zero
//     columns around the data), and the horizontal transpose writes the
//     folded window to scratch, column by column (lanes take rows, so the
//     stores of a wave cover consecutive addresses).  It also records each
//     fragment's radius.
//  2. fov_adj_sum_kernel — one workgroup per output tile (the fragment grid)
//     adds up the windows of every fragment that reaches it, in a fixed
//     order (lanes test the candidate fragments, a ballot lists the hits),
//     reading window columns with buffer loads, and stores the tile along
//     rows through an LDS transpose.
// Both transposes are the forward's register-window correlations, run over
// the band of taps that meet the fragment.
#include "adjoint.h"

#include <hip/hip_runtime.h>

#include <algorithm>

#include "conv.h"

namespace fov {

namespace {

constexpr int kPadA = 12;  // zero columns before a window row (horizontal transpose)

// Folded window of fragment F at radius r: frame rows [y0, y1), columns [x0, x1].
struct Window {
    int y0, y1, x0, x1;
};

__device__ __forceinline__ Window window_of(const Frag& F, int r, int h, int w) {
    Window v;
    v.y0 = max(F.ya - r, 0);
    v.y1 = min(F.ya + F.bh + r, h);
    v.x0 = max(F.xa - r, 0);
    v.x1 = min(F.xa + F.bw - 1 + r, w - 1);
    return v;
}

// Blur strength of fragment (bx, by), local index lb, of a frame: from the sigma map or from the
// midpoint's eccentricity (Sec. 2).
__device__ __forceinline__ double fragment_sigma(const FrameParams& fp, int lb, int bx, int by) {
    return fp.sigma_map ? clip_map_sigma((double)as_global(fp.sigma_map)[lb], fp.cap) : fragment_sigma_ramp(fp, bx, by);
}

// Fragment gid of the launch, its frame read from the kernel arguments (ARGS: launches of up to
// kArgFrames frames) or from the device table.
template <bool ARGS>
__device__ __forceinline__ Frag frag_of(const FwdLaunch& a, const FrameDesc* __restrict__ table,
                                        const int32_t* __restrict__ prefix, int gid) {
    if constexpr (ARGS) {
        int f = 0;
        while (f + 1 < a.nframes && gid >= a.kprefix[f + 1]) ++f;
        return describe_at(&a.fr[f], a.kprefix[f], gid);
    } else {
        return describe(table, prefix, a.nframes, gid);
    }
}

// The fragment's taps in LDS: V copies (V = 16 / sizeof(T)), copy k holding tap i at element
// k * stride + kAdjWeightLead + k + i (stride a multiple of 4) with zeros around, so that a run of
// taps starting at any tap t >= -kAdjWeightLead + 1 starts on a 16-byte boundary in one of them and
// is read with 16-byte loads.
template <typename T>
__device__ __forceinline__ const T* taps_from(const T* taps, int stride, int t) {
    constexpr int V = 16 / sizeof(T);
    const int k = (-t) & (V - 1);
    return static_cast<const T*>(__builtin_assume_aligned(taps + k * stride + kAdjWeightLead + k + t, 16));
}

// Transposed window of fragment gid into scratch[gid][c][x - x0][y - ya + window_lead(r)]
// (column-major, column stride s.sh) for the frame columns x0..x1 and rows y0..y1-1 of its folded
// window: the fragment's own rows start on a 128-byte boundary, and so do those of the tiles above
// and below when the block size is a multiple of 128 bytes of elements.  Workgroup
// q takes fragment q / csplit and its channel share q % csplit (csplit workgroups per fragment).
// GV: gradient values a thread holds per channel (bh * bw <= 256 GV).
template <typename T, int GV, bool ARGS>
__global__ __launch_bounds__(kThreads) void fov_adj_window_kernel(const FwdLaunch a, const AdjShape s,
                                                                  const FrameDesc* __restrict__ table,
                                                                  const int32_t* __restrict__ prefix,
                                                                  int32_t* __restrict__ radius, T* __restrict__ scratch,
                                                                  int csplit) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int V = 16 / sizeof(T);  // elements per aligned 16-byte LDS load
    const int PB = s.pitch_b, PAD = s.pad_b, P = s.pitch_a;
    T* taps = reinterpret_cast<T*>(smem);  // V shifted copies of the taps (taps_from)
    T* G = taps + s.tap_elems;             // [bmax columns][PB rows]: one channel's gradient, rows PAD..
    T* R = G + (size_t)s.bmax * PB;        // [s.rows_r rows][P]: vertical transpose of a run of window
                                           // rows, columns kPadA..
    __shared__ double part_of_wave[kThreads / 64];
    const int gid = blockIdx.x / csplit, share = blockIdx.x - gid * csplit;
    const Frag F = frag_of<ARGS>(a, table, prefix, gid);
    const FrameDesc& d = *F.fd;
    const int per = (s.cmax + csplit - 1) / csplit;
    const int c_begin = share * per, c_end = min(d.c, c_begin + per);
    if (c_begin >= c_end) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const global_ptr<const T> g = as_global(static_cast<const T*>(d.in));
    // One channel's gradient in registers, thread values i = tid + 256 k at row i / bmax, column
    // i % bmax (lanes along a row: coalesced reads); the next channel's loads are issued while this
    // channel is transposed.
    constexpr int kGv = GV;
    T gv[kGv];
    int gy[kGv], gx[kGv];  // row and column of each value (-1: none)
#pragma unroll
    for (int k = 0; k < kGv; ++k) {
        const int i = tid + k * kThreads;
        const int py = div_by(i, s.bdiv), x = i - py * s.bmax;
        const bool in = x < F.bw && py < F.bh;
        gy[k] = in ? py : -1;
        gx[k] = x;
    }
    auto load_g = [&](int c) {
#pragma unroll
        for (int k = 0; k < kGv; ++k)
            if (gy[k] >= 0)
                gv[k] = g[(int64_t)c * d.isc + (int64_t)(F.ya + gy[k]) * d.ish + (int64_t)(F.xa + gx[k]) * d.isw];
    };
    load_g(c_begin);
    // Radius and normalised taps of the fragment (its sigma from the midpoint's eccentricity, Sec. 2;
    // Eq. 1 cut at 3 sigma), as the forward's plan computes them.
    const FrameParams& fp = d.p;
    const double sigma = fragment_sigma(fp, F.lb, F.bx, F.by);
    const int r = min(radius_of(sigma), a.r_cap);
    const int N = 2 * r + 1;
    if (share == 0 && tid == 0) radius[gid] = r;  // for the sum kernel
    const double inv = r > 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
    double part = 0.0, mine = 0.0;
    for (int j = tid; j < N; j += kThreads) {
        const double k = (double)(j - r);
        const double e = exp(-(k * k) * inv);
        part += e;
        if (j == tid) mine = e;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) part_of_wave[wave] = part;
    const Window win = window_of(F, r, d.h, d.w);
    const int RT = win.y1 - win.y0;
    const int CH = s.rows_r;  // window rows transposed per run (a multiple of 4)
    // Zeros: the taps' padding, and the staged gradient and transposed rows (whose data cells every
    // channel and run overwrite).
    for (int k = 0; k < V; ++k)
        for (int j = tid; j < s.tap_stride; j += kThreads) {
            const int t = j - kAdjWeightLead - k;
            if (t < 0 || t >= N) taps[k * s.tap_stride + j] = (T)0;
        }
    {
        using V16 = __attribute__((ext_vector_type(4))) uint32_t;
        V16* z = reinterpret_cast<V16*>(G);
        const int n16 = (s.bmax * PB + min(RT, CH) * P) / V;
        for (int i = tid; i < n16; i += kThreads) z[i] = V16{0, 0, 0, 0};
    }
    __syncthreads();
    part = 0.0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) part += part_of_wave[q];
    for (int j = tid; j < N; j += kThreads) {
        const double k = (double)(j - r);
        const T v = (T)((j == tid ? mine : exp(-(k * k) * inv)) / part);
#pragma unroll
        for (int c = 0; c < V; ++c) taps[c * s.tap_stride + kAdjWeightLead + c + j] = v;
    }
    const T* __restrict__ w = taps + kAdjWeightLead;  // copy 0, w[i] = tap i (i = t + r)
    T* dst0 = scratch + (size_t)gid * s.cmax * s.sw * s.sh;
    const int G8 = (win.x1 - win.x0 + kPH) / kPH;
    // Barriers: one before each run's vertical transpose (the staged gradient and the taps are
    // visible; the previous run's rows are no longer read) and one after it (the rows are written;
    // the gradient is no longer read, so the next channel may be staged).
    for (int c = c_begin; c < c_end; ++c) {
        // the fragment's gradient, column-major
#pragma unroll
        for (int k = 0; k < kGv; ++k)
            if (gy[k] >= 0) G[gx[k] * PB + PAD + gy[k]] = gv[k];
        if (c + 1 < c_end) load_g(c + 1);
        for (int cr0 = win.y0; cr0 < win.y1; cr0 += CH) {
        const int rows = min(CH, win.y1 - cr0);  // window rows cr0 .. cr0 + rows - 1 in this run
        const int ngroups = (rows + kPV - 1) / kPV;
        const int ntask_v = s.bmax * ngroups;  // task i: column i % bmax, rows cr0 + 4 (i / bmax) .. +3
        __syncthreads();
        // Vertical transpose Fold_y V^T g into R: a wave's 64 tasks share one band of taps (the taps
        // that meet the fragment's rows from some row of the wave).
        for (int i0 = wave * 64; i0 < ntask_v; i0 += kThreads) {
            const int gA = div_by(i0, s.bdiv), gB = min(div_by(i0 + 63, s.bdiv), ngroups - 1);
            const int ymin = cr0 + kPV * gA, ymax = min(cr0 + kPV * gB + kPV - 1, cr0 + rows - 1);
            int t_lo = max(-r, F.ya - ymax);
            const int t_hi = min(r, F.ya + F.bh - 1 - ymin);
            if (t_lo <= t_hi) t_lo -= (cr0 + kPV * gA + t_lo - F.ya + PAD) & (V - 1);  // aligned start
            const int i = i0 + lane;
            const int gr = div_by(i, s.bdiv), x = i - gr * s.bmax;
            if (x >= F.bw || gr >= ngroups) continue;
            const int y0 = cr0 + kPV * gr;
            T acc[kPV];
#pragma unroll
            for (int p = 0; p < kPV; ++p) acc[p] = 0;
            const T* col = G + x * PB + PAD - F.ya;  // col[y]: the gradient at frame row y (zero outside)
            if (t_lo <= t_hi) vconv(acc, col + y0 + t_lo, t_hi - t_lo + 1, taps_from(taps, s.tap_stride, t_lo + r));
            if (y0 == 0) {  // row 0 collects the taps off the top edge
                T cdf = 0, corr = 0;
                for (int m = -r; m <= -F.ya - 1; ++m) {
                    cdf += w[m + r];
                    const int py = -m - 1;
                    if (py < F.ya + F.bh) corr = fma(cdf, col[py], corr);
                }
                acc[0] += corr;
            }
            const int pr = d.h - 1 - y0;  // row h-1 collects those off the bottom edge
            if (pr >= 0 && pr < kPV) {
                T cdf = 0, corr = 0;
                for (int m = -r; m <= -1; ++m) {
                    cdf += w[m + r];
                    const int py = m + d.h;
                    if (py >= F.ya && py < F.ya + F.bh) corr = fma(cdf, col[py], corr);
                }
#pragma unroll
                for (int p = 0; p < kPV; ++p)
                    if (p == pr) acc[p] += corr;
            }
            T* rr = R + (y0 - cr0) * P + kPadA + x;
#pragma unroll
            for (int p = 0; p < kPV; ++p)
                if (y0 + p < cr0 + rows) rr[p * P] = acc[p];
        }
        __syncthreads();
        // Horizontal transpose Fold_x H^T of the window rows into scratch: lanes take rows, a wave
        // shares one group of 8 output columns, so the taps that meet the fragment form one
        // wave-uniform range.
        T* dstc = dst0 + (size_t)c * s.sw * s.sh + (cr0 - F.ya + window_lead(r, (int)sizeof(T)));
        for (int ch = 0; ch * 64 < rows; ++ch)
        for (int gi = wave; gi < G8; gi += kThreads / 64) {
            const int X = win.x0 + gi * kPH;
            // taps t with X + p + t inside the fragment for some p in 0..7
            int t_lo = max(-r, F.xa - X - (kPH - 1));
            const int t_hi = min(r, F.xa + F.bw - 1 - X);
            const int row = ch * 64 + lane;
            if (row >= rows) continue;
            const T* rr = R + row * P + kPadA - F.xa;  // rr[x]: this row at frame column x
            T acc[kPH];
#pragma unroll
            for (int p = 0; p < kPH; ++p) acc[p] = 0;
            if (t_lo <= t_hi) {
                t_lo -= (X + t_lo - F.xa + kPadA) & (V - 1);  // aligned window start; taps below -r are zero
                hconv(acc, rr + X + t_lo, t_hi - t_lo + 1, taps_from(taps, s.tap_stride, t_lo + r));
            }
            if (win.x0 == 0 && gi == 0) {  // column 0 collects the taps that fell off the left edge
                T cdf = 0, corr = 0;
                for (int m = -r; m <= -F.xa - 1; ++m) {
                    cdf += w[m + r];
                    const int x = -m - 1;
                    if (x < F.xa + F.bw) corr = fma(cdf, rr[x], corr);
                }
                acc[0] += corr;
            }
            const int jr = d.w - 1 - X;
            if (win.x1 == d.w - 1 && jr >= 0 && jr < kPH) {  // column w-1 collects those off the right edge
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
            T* dst = dstc + (size_t)(X - win.x0) * s.sh + row;
#pragma unroll
            for (int p = 0; p < kPH; ++p)
                if (X + p <= win.x1) dst[(size_t)p * s.sh] = acc[p];
        }
        }
    }
}

// Output tile gid: grad_in over the fragment's rectangle, the sum of the windows of every fragment
// that reaches it, in a fixed order (fragment rows, then columns).  Pixel i of the tile is column
// i / bh, row i % bh, so the lanes of a wave read consecutive rows of a window column.  Up to
// kSumCh channels are summed together, and the windows are read kSumBatch at a time, all their loads
// in flight before the values are added in order (PIX: pixels per thread, bh * bw <= 256 PIX).
constexpr int kSumCh = 3;
// Windows in flight per batch, sized so that the loaded values stay within the register budget of
// four waves per SIMD.
template <typename T, int PIX>
constexpr int sum_batch() {
    return PIX * (int)sizeof(T) <= 16 ? 4 : (PIX * (int)sizeof(T) <= 64 ? 2 : 1);
}

struct SumNb {
    int b;      // fragment
    int ybase;  // frame row of the first element of its window columns
    Window w;
};

// Raw buffer descriptor (dword 3 as gfx9 expects for untyped access).
constexpr int kBufferWord3 = 0x00020000;
// Byte offset past any window plane: a buffer load there returns 0.
constexpr uint32_t kOutside = 0x7fffffffu;

template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t rsrc, uint32_t voff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)voff, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)voff, 0, 0));
}

// The values of window n at this thread's pixels, channels c0 .. c0 + kSumCh - 1 (zero outside the
// window and for channels >= c0 + cc): one buffer descriptor per channel plane of the window, so a
// pixel outside it reads 0 through the descriptor's range check.
template <typename T, int PIX>
__device__ __forceinline__ void load_window(T (&v)[kSumCh][PIX], const SumNb& n, const T* __restrict__ scratch,
                                            const AdjShape& s, int c0, int cc, const int (&px)[PIX],
                                            const int (&py)[PIX]) {
    const uint32_t wx = (uint32_t)(n.w.x1 - n.w.x0), wy = (uint32_t)(n.w.y1 - n.w.y0);
    uint32_t voff[PIX];
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const uint32_t dx = (uint32_t)(px[k] - n.w.x0), dy = (uint32_t)(py[k] - n.w.y0);
        voff[k] = (dx <= wx && dy < wy) ? (dx * (uint32_t)s.sh + (uint32_t)(py[k] - n.ybase)) * (uint32_t)sizeof(T)
                                        : kOutside;
    }
    const int plane = s.sw * s.sh;
#pragma unroll
    for (int ch = 0; ch < kSumCh; ++ch) {
        if (ch < cc) {
            const T* src = scratch + ((size_t)n.b * s.cmax + c0 + ch) * plane;
            const __amdgpu_buffer_rsrc_t rsrc =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(src), 0, plane * (int)sizeof(T), kBufferWord3);
#pragma unroll
            for (int k = 0; k < PIX; ++k) v[ch][k] = buffer_load<T>(rsrc, voff[k]);
        } else {
#pragma unroll
            for (int k = 0; k < PIX; ++k) v[ch][k] = (T)0;
        }
    }
}

__device__ __forceinline__ int lane_value(int v, int j) { return __builtin_amdgcn_readlane(v, j); }

template <typename T, int PIX, bool ARGS>
__global__ __launch_bounds__(kThreads) void fov_adj_sum_kernel(const FwdLaunch a, const AdjShape s,
                                                               const FrameDesc* __restrict__ table,
                                                               const int32_t* __restrict__ prefix,
                                                               const int32_t* __restrict__ radius,
                                                               const T* __restrict__ scratch) {
    const int gid = blockIdx.x;
    const Frag Q = frag_of<ARGS>(a, table, prefix, gid);
    const FrameDesc& d = *Q.fd;
    const FrameParams& fp = d.p;
    const int nbx = fp.nbx, nby = d.nby;
    const int first = gid - Q.lb;
    const int K = (a.r_cap + fp.block - 1) / fp.block;  // fragments within reach on each side
    const int by_lo = max(Q.by - K, 0), by_hi = min(Q.by + K, nby - 1);
    const int bx_lo = max(Q.bx - K, 0), bx_hi = min(Q.bx + K, nbx - 1);
    const int nx = bx_hi - bx_lo + 1, ncand = nx * (by_hi - by_lo + 1);
    const float rnx = 1.0f / (float)nx;  // candidate j is row j / nx of the neighbourhood
    const int lane = threadIdx.x & 63;
    const int B = fp.block;
    int px[PIX], py[PIX];  // frame column and row of each pixel (-1: none)
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
        const int i = threadIdx.x + k * kThreads;
        const int col = div_by(i, s.bdiv), row = i - col * s.bmax;
        const bool in = col < Q.bw && row < Q.bh;
        px[k] = in ? Q.xa + col : -1;
        py[k] = in ? Q.ya + row : -1;
    }
    const global_ptr<T> out = as_global(static_cast<T*>(d.out));
    extern __shared__ __align__(16) unsigned char smem[];
    T* tile = reinterpret_cast<T*>(smem);
    const int LP = s.bmax + 1;
    constexpr int kSumBatch = sum_batch<T, PIX>();
    for (int c0 = 0; c0 < d.c; c0 += kSumCh) {
        const int cc = min(kSumCh, d.c - c0);
        T acc[kSumCh][PIX];
#pragma unroll
        for (int ch = 0; ch < kSumCh; ++ch)
#pragma unroll
            for (int k = 0; k < PIX; ++k) acc[ch][k] = 0;
        for (int j0 = 0; j0 < ncand; j0 += 64) {
            // Candidates j0 .. j0 + 63 (row-major over the fragments within reach), one per lane: the
            // ballot of those whose window meets the tile lists them in the fixed summation order.
            const int j = j0 + lane;
            int b = 0, y0 = 0, y1 = 0, x0 = 0, x1 = 0, yb = 0;
            bool hit = false;
            if (j < ncand) {
                const int jy = (int)(((float)j + 0.5f) * rnx);
                const int by = by_lo + jy, bx = bx_lo + (j - jy * nx);
                const int lb = by * nbx + bx;
                b = first + lb;
                const int rb = radius[b];
                // its folded window (as window_of gives it for that fragment)
                const int X0 = fp.origin_x + bx * B, Y0 = fp.origin_y + by * B;
                x0 = max(X0 - rb, 0);
                x1 = min(X0 + B - 1 + rb, d.w - 1);
                y0 = max(Y0 - rb, 0);
                y1 = min(Y0 + B + rb, d.h);
                yb = max(Y0, 0) - window_lead(rb, (int)sizeof(T));
                hit = x1 >= Q.xa && x0 < Q.xa + Q.bw && y1 > Q.ya && y0 < Q.ya + Q.bh;
            }
            uint64_t m = __ballot(hit);
            while (m) {
                // the next kSumBatch of them: all their loads in flight, then added in order
                SumNb nb[kSumBatch];
                int cnt = 0;
#pragma unroll
                for (int q = 0; q < kSumBatch; ++q) {
                    if (m) {
                        const int l = __builtin_ctzll(m);
                        m &= m - 1;
                        nb[q].b = lane_value(b, l);
                        nb[q].ybase = lane_value(yb, l);
                        nb[q].w.y0 = lane_value(y0, l);
                        nb[q].w.y1 = lane_value(y1, l);
                        nb[q].w.x0 = lane_value(x0, l);
                        nb[q].w.x1 = lane_value(x1, l);
                        ++cnt;
                    }
                }
                T v[kSumBatch][kSumCh][PIX];
#pragma unroll
                for (int q = 0; q < kSumBatch; ++q)
                    if (q < cnt) load_window(v[q], nb[q], scratch, s, c0, cc, px, py);
#pragma unroll
                for (int q = 0; q < kSumBatch; ++q)
                    if (q < cnt) {
#pragma unroll
                        for (int ch = 0; ch < kSumCh; ++ch)
#pragma unroll
                            for (int k = 0; k < PIX; ++k) acc[ch][k] += v[q][ch][k];
                    }
            }
        }
        // Through LDS (tile[ch][row][col], pitch bmax + 1) so that the stores run along rows.
        if (c0 > 0) __syncthreads();  // the previous channels' tile is read
#pragma unroll
        for (int ch = 0; ch < kSumCh; ++ch)
#pragma unroll
            for (int k = 0; k < PIX; ++k)
                if (ch < cc && px[k] >= 0) tile[(ch * s.bmax + py[k] - Q.ya) * LP + px[k] - Q.xa] = acc[ch][k];
        __syncthreads();
        int tx = threadIdx.x;
        asm volatile("" : "+v"(tx));  // store addresses computed here, not held through the sums
#pragma unroll
        for (int k = 0; k < PIX; ++k) {
            const int i = tx + k * kThreads;
            const int row = div_by(i, s.bdiv), col = i - row * s.bmax;
            if (row >= Q.bh || col >= Q.bw) continue;
#pragma unroll
            for (int ch = 0; ch < kSumCh; ++ch)
                if (ch < cc)
                    out[(int64_t)(c0 + ch) * d.osc + (int64_t)(Q.ya + row) * d.osh + (int64_t)(Q.xa + col) * d.osw] =
                        tile[(ch * s.bmax + row) * LP + col];
        }
    }
}

template <typename T, int GV, bool ARGS>
fov_status launch_kernels(const FwdLaunch& a, const AdjShape& s, int32_t* radius, T* sc, hipStream_t stream,
                          size_t lds_limit) {
    const auto kw = fov_adj_window_kernel<T, GV, ARGS>;
    fov_status st;
    if ((st = allow_dyn_lds((const void*)kw, lds_limit)) != FOV_OK) return st;
    // one window workgroup per fragment and channel (per fragment if the grid would be too large)
    const int csplit = (int64_t)a.nfrag * s.cmax * kThreads < ((int64_t)1 << 32) ? s.cmax : 1;
    hipLaunchKernelGGL(kw, dim3(a.nfrag * csplit), dim3(kThreads), adjoint_lds(s, sizeof(T)), stream, a, s,
                       (const FrameDesc*)a.table, (const int32_t*)a.prefix, radius, sc, csplit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint window kernel launch");
    const auto ks = fov_adj_sum_kernel<T, GV, ARGS>;
    const size_t sum_lds = (size_t)kSumCh * s.bmax * (s.bmax + 1) * sizeof(T);
    if (sum_lds + 64 > lds_limit) return set_error(FOV_ERANGE, "adjoint output tile does not fit in LDS");
    if ((st = allow_dyn_lds((const void*)ks, lds_limit)) != FOV_OK) return st;
    hipLaunchKernelGGL(ks, dim3(a.nfrag), dim3(kThreads), sum_lds, stream, a, s,
                       (const FrameDesc*)a.table, (const int32_t*)a.prefix, (const int32_t*)radius, (const T*)sc);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint sum kernel launch");
    return FOV_OK;
}

template <typename T>
fov_status launch_typed(const FwdLaunch& a, const AdjShape& s, int32_t* radius, void* scratch, hipStream_t stream,
                        size_t lds_limit) {
    // values per thread: 4 for fragments of at most 32 x 32 pixels, else kMaxBlock^2 / kThreads
    constexpr int kBig = kMaxBlock * kMaxBlock / kThreads;
    const bool small = s.bmax * s.bmax <= 4 * kThreads;
    T* sc = static_cast<T*>(scratch);
    if (a.from_args)
        return small ? launch_kernels<T, 4, true>(a, s, radius, sc, stream, lds_limit)
                     : launch_kernels<T, kBig, true>(a, s, radius, sc, stream, lds_limit);
    return small ? launch_kernels<T, 4, false>(a, s, radius, sc, stream, lds_limit)
                 : launch_kernels<T, kBig, false>(a, s, radius, sc, stream, lds_limit);
}

}  // namespace

AdjShape adjoint_shape(int es, int r_cap, int bmax, int cmax) {
    AdjShape s;
    s.bmax = bmax;
    s.sw = bmax + 2 * r_cap;
    s.sh = round_up(bmax + r_cap + window_lead(r_cap, es), 128 / es);
    s.cmax = cmax;
    s.pitch_a = tile_pitch(bmax + kPadA + 7, es);
    // rows one wave's tasks span in the vertical transpose, minus one
    const int span = std::min(kPV * (63 / bmax + 1) + kPV - 1, bmax + 2 * r_cap - 1);
    s.pad_b = round_up(span + 4, 4);
    s.pitch_b = inter_pitch(bmax + 2 * s.pad_b, es);
    s.tap_stride = round_up(2 * r_cap + 1 + kAdjWeightLead + 8, 4);
    s.tap_elems = (16 / es) * s.tap_stride;
    s.bdiv = div_magic((uint32_t)bmax);
    // window rows transposed per run: the whole window when the LDS stays within kAdjLdsBudget,
    // else as many rows (a multiple of 4, at least 4) as fit beside the staged gradient
    const size_t g = ((size_t)s.tap_elems + (size_t)bmax * s.pitch_b) * es, row = (size_t)s.pitch_a * es;
    const int fit = g + 4 * row <= kAdjLdsBudget ? (int)((kAdjLdsBudget - g) / row) / 4 * 4 : 4;
    s.rows_r = std::min(round_up(s.sw, 4), fit);
    return s;
}

size_t adjoint_lds(const AdjShape& s, int es) {
    return ((size_t)s.tap_elems + (size_t)s.bmax * s.pitch_b + (size_t)s.rows_r * s.pitch_a) * es;
}

size_t adjoint_scratch_elems(const AdjShape& s, int nfrag) { return (size_t)nfrag * s.cmax * s.sw * s.sh; }

fov_status launch_adjoint(const FwdLaunch& a, const AdjShape& s, int es, int32_t* radius, void* scratch,
                          hipStream_t stream, size_t lds_limit) {
    if (a.nfrag <= 0) return FOV_OK;
    if (adjoint_lds(s, es) + 64 > lds_limit) return set_error(FOV_ERANGE, "adjoint tiles do not fit in LDS");
    return es == 8 ? launch_typed<double>(a, s, radius, scratch, stream, lds_limit)
                   : launch_typed<float>(a, s, radius, scratch, stream, lds_limit);
}

}  // namespace fov
