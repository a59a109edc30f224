// Forward block-wise foveation for gfx950.
//
// Three launches per batch of frames on the caller's stream:
//
//  1. fov_plan_weights_kernel — one wavefront per fragment: the fragment's
//     sigma from its midpoint's eccentricity (Sec. 2, Fig. 1), radius
//     r = ceil(3 sigma) and the normalised taps w_k = exp(-k^2/(2 sigma^2)) / sum
//     (Eq. 1 cut at 3 sigma, Appendix "Methods"), summed with wavefront
//     shuffles, written to the plan workspace.
//
//  2. fov_order_kernel — a counting sort of fragments by decreasing radius
//     (costliest first), dealt within each radius in angular arcs to the
//     eight XCDs: the dispatch order of the main kernel.
//
//  3. fov_fwd_kernel — one workgroup per work item (Alg. 1): the padded
//     tile (fragment plus r on each side, clamp-to-edge) is staged into LDS
//     with row-coalesced loads, 8-bit input as 16-bit integers; a horizontal
//     pass writes the fp32 intermediate into LDS; a vertical pass produces the
//     fragment (Appendix "Workload of the Block", "Shared Memory").  Each
//     thread computes 8 (horizontal) or 4 (vertical) outputs and slides the
//     filter window through registers (the register reuse of Appendix "Data
//     Reuse"); the work item copies its weights to LDS and both passes read
//     them as broadcast LDS loads.  For 8-bit input the horizontal pass adds
//     the two samples that share a weight (the taps are symmetric) exactly,
//     two sums per 32-bit integer add, before the FP32 multiply-add.  A
//     fragment with r = 0 is copied.
//
// Every output sums its taps in the same order (k = -r .. r; for 8-bit input
// the horizontal pass goes k = 0, then the pairs +-1 .. +-r) whatever the
// strip height, output tile split or dispatch mode, so results do not depend
// on tuning choices.
#include "forward.h"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "conv.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace fov {

namespace {

struct Geom {
    int N;   // taps, 2r+1
    int G;   // horizontal-pass column groups
    int GV;  // vertical-pass row groups
    int TW;  // staged tile columns (8G + 2r)
    int TH;  // staged tile rows = intermediate rows (4GV + 2r)
};

__host__ __device__ inline Geom geom(int r, int bw, int bh) {
    Geom g;
    g.N = 2 * r + 1;
    g.G = (bw + kPH - 1) / kPH;
    g.GV = (bh + kPV - 1) / kPV;
    g.TW = g.G * kPH + g.N - 1;
    g.TH = g.GV * kPV + g.N - 1;
    return g;
}

// ---- element conversions ----------------------------------------------------------------------
template <typename TS, typename TIn>
__device__ __forceinline__ TS to_stage(TIn v) { return (TS)v; }

template <typename TOut, typename TC>
__device__ __forceinline__ TOut to_out(TC v) { return (TOut)v; }
template <>
__device__ __forceinline__ uint8_t to_out<uint8_t, float>(float v) {
    v = rintf(v);  // round half to even
    v = __builtin_amdgcn_fmed3f(v, 0.0f, 255.0f);  // clamp to [0, 255] (the value is never NaN)
    return (uint8_t)v;
}

template <typename TOut, typename TIn>
__device__ __forceinline__ TOut copy_out(TIn v) { return (TOut)v; }

// ---- staging of the padded tile ---------------------------------------------------------------
// The tile is staged into LDS in strips of at most kStripMax rows.  Each strip
// is loaded in two halves: issue() starts the global loads into registers
// (lanes walk columns, so loads coalesce along x; wave w owns rows w, w+4,
// ...), commit() converts the values and writes them to LDS.  The kernel
// issues strip k+1 before computing strip k, so load latency hides behind
// arithmetic.  Columns beyond the prefetched chunks are loaded and written
// inside commit().
constexpr int kStripMax = 64;
// Bytes of LDS before the tile: the symmetric horizontal pass may read (and ignore) up to three
// samples before a row's first one.
constexpr int kTileLead = 16;
constexpr int kRowsPerWave = kStripMax / (kThreads / 64);

template <typename TIn, typename TS>
struct Stager {
    static constexpr int KB = 2;  // prefetched 64-column chunks
    TIn v[kRowsPerWave][KB];
    uint32_t coff[KB];
    bool cv[KB];
    const TIn* plane;
    int64_t ish, isw;
    int y0, rows, h, w, x_first, TW;

    __device__ __forceinline__ void setup(int x_first_, int TW_, int w_, int64_t isw_, int64_t ish_, int h_,
                                          const TIn*, uint32_t) {
        x_first = x_first_; TW = TW_; w = w_; isw = isw_; ish = ish_; h = h_;
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int tx = kb * 64 + lane;
            cv[kb] = tx < TW;
            coff[kb] = (uint32_t)clampi(x_first + tx, 0, w - 1) * (uint32_t)isw;
        }
    }
    __device__ __forceinline__ void issue(const TIn* plane_, int y0_, int rows_) {
        plane = plane_; y0 = y0_; rows = rows_;
        const int wave = wave_id();
#pragma unroll
        for (int rb = 0; rb < kRowsPerWave; ++rb) {
            const int ty = wave + rb * (kThreads / 64);
            if (ty < rows) {
                const TIn* rp = plane + (int64_t)clampi(y0 + ty, 0, h - 1) * ish;
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    if (cv[kb]) v[rb][kb] = rp[coff[kb]];
            }
        }
    }
    __device__ __forceinline__ void commit(TS* tile, int TP) {
        const int wave = wave_id(), lane = threadIdx.x & 63;
#pragma unroll
        for (int rb = 0; rb < kRowsPerWave; ++rb) {
            const int ty = wave + rb * (kThreads / 64);
            if (ty < rows) {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    if (cv[kb]) tile[ty * TP + kb * 64 + lane] = to_stage<TS, TIn>(v[rb][kb]);
            }
        }
        for (int k0 = 64 * KB; k0 < TW; k0 += 64) {
            const int tx = k0 + lane;
            if (tx >= TW) continue;
            const uint32_t co = (uint32_t)clampi(x_first + tx, 0, w - 1) * (uint32_t)isw;
            for (int ty = wave; ty < rows; ty += kThreads / 64)
                tile[ty * TP + tx] = to_stage<TS, TIn>(plane[(int64_t)clampi(y0 + ty, 0, h - 1) * ish + co]);
        }
    }
};

// 8-bit input staged as 16-bit integers, two columns per lane and one 32-bit
// LDS write per pair (b1 << 16 | b0).  Read as fp16, such a half is the
// subnormal b * 2^-24, which the symmetric horizontal pass multiplies by taps
// scaled by 2^24.  One 128-column chunk is prefetched.  Bytes are read with
// buffer loads over the frame (a descriptor covering its bytes): each lane's
// two column offsets are fixed for the fragment and a row's offset is a
// wave-uniform scalar, so no per-row address arithmetic runs on the vector
// unit; reads past the descriptor's range would return 0.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half2_t bytes_to_half2(uint32_t b0, uint32_t b1) {
    return __builtin_bit_cast(half2_t, (b1 << 16) | b0);
}

// Raw buffer descriptor (dword 3 as gfx9 expects for untyped access).
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ uint32_t load_byte(__amdgpu_buffer_rsrc_t rsrc, uint32_t voff, uint32_t soff) {
    return (uint32_t)(uint8_t)__builtin_amdgcn_raw_buffer_load_b8(rsrc, (int)voff, (int)soff, 0);
}

template <>
struct Stager<uint8_t, _Float16> {
    uint32_t b0[kRowsPerWave], b1[kRowsPerWave];
    uint32_t c0, c1;
    bool cv;
    __amdgpu_buffer_rsrc_t rsrc;
    const uint8_t* base;
    uint32_t poff, ish;
    uint32_t isw;
    int y0, rows, h, w, x_first, TW;

    // base: the frame's first byte; span: bytes from base to its last byte + 1 (< 2^31)
    __device__ __forceinline__ void setup(int x_first_, int TW_, int w_, int64_t isw_, int64_t ish_, int h_,
                                          const uint8_t* base_, uint32_t span) {
        x_first = x_first_; TW = TW_; w = w_; isw = (uint32_t)isw_; ish = (uint32_t)ish_; h = h_;
        base = base_;
        rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base_), 0, (int)span, kBufferWord3);
        const int tx = 2 * (threadIdx.x & 63);  // tx + 1 < TP always
        cv = tx < TW;
        c0 = (uint32_t)clampi(x_first + tx, 0, w - 1) * isw;
        c1 = (uint32_t)clampi(x_first + tx + 1, 0, w - 1) * isw;
    }
    __device__ __forceinline__ void issue(const uint8_t* plane_, int y0_, int rows_) {
        poff = (uint32_t)(plane_ - base);
        y0 = y0_; rows = rows_;
        if (!cv) return;  // one lane predicate for all rows (not one exec-mask region per row)
        const int wave = wave_id();
        if (y0 >= 0 && y0 + rows <= h) {
            // strip inside the frame: row offsets step by 4 rows, no clamping
            const uint32_t s0 = poff + (uint32_t)(y0 + wave) * ish, step = (uint32_t)(kThreads / 64) * ish;
            if (rows == kStripMax) {  // full strip: every row of every wave
#pragma unroll
                for (int rb = 0; rb < kRowsPerWave; ++rb) {
                    b0[rb] = load_byte(rsrc, c0, s0 + rb * step);
                    b1[rb] = load_byte(rsrc, c1, s0 + rb * step);
                }
                return;
            }
#pragma unroll
            for (int rb = 0; rb < kRowsPerWave; ++rb)
                if (wave + rb * (kThreads / 64) < rows) {
                    b0[rb] = load_byte(rsrc, c0, s0 + rb * step);
                    b1[rb] = load_byte(rsrc, c1, s0 + rb * step);
                }
            return;
        }
#pragma unroll
        for (int rb = 0; rb < kRowsPerWave; ++rb) {
            const int ty = wave + rb * (kThreads / 64);
            if (ty < rows) {
                const uint32_t soff = poff + (uint32_t)clampi(y0 + ty, 0, h - 1) * ish;
                b0[rb] = load_byte(rsrc, c0, soff);
                b1[rb] = load_byte(rsrc, c1, soff);
            }
        }
    }
    __device__ __forceinline__ void commit(_Float16* tile, int TP) {
        const int wave = wave_id(), lane = threadIdx.x & 63;
        if (cv) {
            half2_t* dst = reinterpret_cast<half2_t*>(tile + wave * TP + 2 * lane);
            const int step = (kThreads / 64) * TP / 2;  // half2 elements per 4 rows (TP is even)
            if (rows == kStripMax) {
#pragma unroll
                for (int rb = 0; rb < kRowsPerWave; ++rb) dst[rb * step] = bytes_to_half2(b0[rb], b1[rb]);
            } else {
#pragma unroll
                for (int rb = 0; rb < kRowsPerWave; ++rb)
                    if (wave + rb * (kThreads / 64) < rows) dst[rb * step] = bytes_to_half2(b0[rb], b1[rb]);
            }
        }
        for (int k0 = 128; k0 < TW; k0 += 128) {
            const int tx = k0 + 2 * lane;
            if (tx >= TW) continue;
            const uint32_t d0 = (uint32_t)clampi(x_first + tx, 0, w - 1) * isw;
            const uint32_t d1 = (uint32_t)clampi(x_first + tx + 1, 0, w - 1) * isw;
            for (int ty = wave; ty < rows; ty += kThreads / 64) {
                const uint32_t soff = poff + (uint32_t)clampi(y0 + ty, 0, h - 1) * ish;
                *reinterpret_cast<half2_t*>(tile + ty * TP + tx) =
                    bytes_to_half2(load_byte(rsrc, d0, soff), load_byte(rsrc, d1, soff));
            }
        }
    }
};

// ---- fragments of a launch ---------------------------------------------------------------------
// Narrow a fragment to output tile `sub` of its L-level split: tiles of
// T = ceil(B / 2^L) pixels a side, row-major, clipped to the fragment and the
// frame.  Returns false for a tile that holds no pixel (ragged splits).
__device__ __forceinline__ bool narrow_to_tile(Frag& F, int L, int sub) {
    if (L == 0) return true;
    const FrameParams& fp = F.fd->p;
    const int B = fp.block, T = (B + (1 << L) - 1) >> L;
    const int sx = sub & ((1 << L) - 1), sy = sub >> L;
    const int X0 = fp.origin_x + F.bx * B, Y0 = fp.origin_y + F.by * B;
    const int x0 = X0 + sx * T, y0 = Y0 + sy * T;
    const int x1 = min(min(x0 + T, X0 + B), F.fd->w), y1 = min(min(y0 + T, Y0 + B), F.fd->h);
    F.xa = max(x0, 0);
    F.ya = max(y0, 0);
    F.bw = x1 - F.xa;
    F.bh = y1 - F.ya;
    return F.bw > 0 && F.bh > 0;
}

// Foveal fragment: copied (Appendix "Workload of the Block").
template <typename TIn, typename TOut>
__device__ __forceinline__ void copy_fragment(const Frag& F, int c_lo, int c_hi) {
    const FrameDesc& d = *F.fd;
    const TIn* in = static_cast<const TIn*>(d.in);
    TOut* out = static_cast<TOut*>(d.out);
    const int wave = wave_id(), lane = threadIdx.x & 63;
    for (int c = c_lo; c < c_hi; ++c)
        for (int y = wave; y < F.bh; y += kThreads / 64)
            for (int x = lane; x < F.bw; x += 64) {
                const TIn v = in[c * d.isc + (int64_t)(F.ya + y) * d.ish + (int64_t)(F.xa + x) * d.isw];
                out[c * d.osc + (int64_t)(F.ya + y) * d.osh + (int64_t)(F.xa + x) * d.osw] = copy_out<TOut, TIn>(v);
            }
}

// ---- main kernel ---------------------------------------------------------------------------------
// One fragment: stage its padded tile strip by strip (the next strip's loads
// in flight while the current one is computed), horizontal pass into the
// column-major intermediate, vertical pass into the output.
template <typename TIn, typename TOut, typename TS, typename TC>
__device__ __forceinline__ void process_fragment(const FwdLaunch& a, int gid, int r, const Frag& F, int c_lo,
                                                 int c_hi, const TC* __restrict__ wts, unsigned char* smem) {
    const FrameDesc& d = *F.fd;
    if (r == 0) {
        copy_fragment<TIn, TOut>(F, c_lo, c_hi);
        return;
    }
    const int tid = threadIdx.x;
    const Geom g = geom(r, F.bw, F.bh);
    const int SR = min(min(a.strip_rows, kStripMax), g.TH);
    // 8-bit input: the symmetric horizontal pass wants each output's centre on a 4-sample group,
    // so the tile starts sh = (-r) mod 4 columns further left.
    constexpr bool kSym = std::is_same<TS, _Float16>::value;
    const int sh = kSym ? ((-r) & 3) : 0;
    const int TW = g.TW + sh;
    const int TP = tile_pitch(TW, sizeof(TS));
    const int IP = inter_pitch(g.TH, sizeof(TC));
    // The fragment's taps are copied to LDS once (read by the passes as broadcast LDS loads, so
    // the inner loops wait on LDS only): w[0 .. N-1] = w_{-r} .. w_r, then for the symmetric
    // pass ws[j] = 2^24 w_{j+1} (j = 0 .. r-1) at a 16-byte boundary (scaled for the 16-bit
    // integer samples, which it reads as fp16 subnormals; the scaling is exact).
    TC* w = reinterpret_cast<TC*>(smem + kTileLead);
    TC* ws = w + round_up(g.N, 4);
    TS* tile = reinterpret_cast<TS*>(smem + kTileLead + tap_lds_bytes(a.r_cap, sizeof(TC)));
    TC* inter = reinterpret_cast<TC*>(reinterpret_cast<unsigned char*>(tile) +
                                      align16((size_t)SR * TP * sizeof(TS)));  // [column][row]
    {
        const TC* __restrict__ wg = wts + (size_t)gid * a.wstride;
        for (int i = tid; i < g.N; i += kThreads) {
            const TC v = wg[i];
            w[i] = v;
            if (kSym && i > r) ws[i - r - 1] = v * kSymScale;
        }
    }
    const TIn* in = static_cast<const TIn*>(d.in);
    const int nst = (g.TH + SR - 1) / SR;
    const int nunits = (c_hi - c_lo) * nst;  // (channel, strip) units, channels c_lo .. c_hi - 1
    // Tasks map to (row, column group) and (column, row group) with shifts: the column groups of a
    // 16-row block and the columns of the vertical pass are padded to powers of two (the padding
    // tasks idle; 32-pixel fragments have none).  LDS offsets stay below 2^24, so their products
    // are 24-bit multiplies.
    const int gsh = ceil_log2(g.G), xsh = ceil_log2(F.bw);
    const uint32_t IPH = (uint32_t)IP * kPH;
    Stager<TIn, TS> st;
    const int64_t span = (int64_t)(d.c - 1) * d.isc + (int64_t)(d.h - 1) * d.ish + (int64_t)(d.w - 1) * d.isw + 1;
    st.setup(F.xa - r - sh, TW, d.w, d.isw, d.ish, d.h, in, (uint32_t)span);
    st.issue(in + c_lo * d.isc, F.ya - r, SR);
    st.commit(tile, TP);
    __syncthreads();
    int cu = 0, sidx = 0;  // the current unit: channel c_lo + cu, strip sidx
    for (int u = 0; u < nunits; ++u) {
        const int c = c_lo + cu;
        const int s0 = sidx * SR, rows = min(SR, g.TH - s0);
        int cn = cu, sn = sidx + 1;  // the next unit
        if (sn == nst) {
            sn = 0;
            ++cn;
        }
        if (u + 1 < nunits) st.issue(in + (c_lo + cn) * d.isc, F.ya - r + sn * SR, min(SR, g.TH - sn * SR));
        // Horizontal pass.  Task t: lanes of a 16-lane group take 16
        // consecutive rows of one column group (conflict-free row reads).
        const int ntask = round_up(rows, 16) << gsh;
        bool four = false;  // 8-bit strips of at most half a workgroup of tasks: 4-output tasks
        if constexpr (kSym) {
            if (ntask <= kThreads / 2) {
                four = true;
                for (int t = tid; t < 2 * ntask; t += kThreads) {
                    const int blk = t >> 4, gi = blk & ((2 << gsh) - 1);
                    const int ty = ((blk >> (gsh + 1)) << 4) | (t & 15);
                    if (ty >= rows || gi >= 2 * g.G) continue;
                    float a4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    const TS* row = tile + __umul24((uint32_t)ty, (uint32_t)TP) + gi * 4;
                    hconv_sym4(a4, row + r + sh, r, w[r] * kSymScale, ws);
                    TC* dst = inter + __umul24((uint32_t)gi, (uint32_t)(4 * IP)) + s0 + ty;
#pragma unroll
                    for (int p = 0; p < 4; ++p) dst[p * IP] = a4[p];
                }
            }
        }
        const int ntask8 = four ? 0 : ntask;
        for (int t = tid; t < ntask8; t += kThreads) {
            const int blk = t >> 4, gi = blk & ((1 << gsh) - 1);
            const int ty = ((blk >> gsh) << 4) | (t & 15);
            if (ty >= rows || gi >= g.G) continue;
            TC acc[kPH];
#pragma unroll
            for (int p = 0; p < kPH; ++p) acc[p] = 0;
            const TS* row = tile + __umul24((uint32_t)ty, (uint32_t)TP) + gi * kPH;
            if constexpr (kSym) hconv_sym(acc, row + r + sh, r, w[r] * kSymScale, ws);
            else hconv(acc, row, g.N, w);
            TC* dst = inter + __umul24((uint32_t)gi, IPH) + s0 + ty;
#pragma unroll
            for (int p = 0; p < kPH; ++p) dst[p * IP] = acc[p];
        }
        __syncthreads();  // the tile is free; the channel's intermediate may be complete
        if (sidx == nst - 1) {
            // Vertical pass over the complete intermediate of channel c.  Output rows step by the
            // row stride from one 64-bit address per task.
            const int64_t osh = d.osh, osw = d.osw;
            const global_ptr<TOut> oc =
                as_global(static_cast<TOut*>(d.out)) + c * d.osc + (int64_t)F.ya * osh + (int64_t)F.xa * osw;
            const int ntv = g.GV << xsh;
            for (int t = tid; t < ntv; t += kThreads) {
                const int x = t & ((1 << xsh) - 1), y0 = (t >> xsh) * kPV;
                if (x >= F.bw) continue;
                TC acc[kPV];
#pragma unroll
                for (int p = 0; p < kPV; ++p) acc[p] = 0;
                vconv(acc, inter + __umul24((uint32_t)x, (uint32_t)IP) + y0, g.N, w);
                global_ptr<TOut> o = oc + (int64_t)x * osw + (int64_t)y0 * osh;
                if ((F.bh & (kPV - 1)) == 0) {  // whole row groups (uniform): no per-row test
#pragma unroll
                    for (int p = 0; p < kPV; ++p) {
                        *o = to_out<TOut, TC>(acc[p]);
                        o += osh;
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < kPV; ++p) {
                        if (y0 + p < F.bh) *o = to_out<TOut, TC>(acc[p]);
                        o += osh;
                    }
                }
            }
        }
        if (u + 1 < nunits) {
            st.commit(tile, TP);
            __syncthreads();  // next strip staged; every thread is past the previous vertical pass
        }
        cu = cn;
        sidx = sn;
    }
}

// Work items are taken from the queue (by decreasing radius, so the costliest
// start first); an item is a whole fragment or, with a split, one output tile
// of it (same radius and taps, its own halo).  PERSIST = false: one workgroup per queue slot,
// the hardware dispatcher hands slots out in order as workgroups retire.
// PERSIST = true: a grid sized to what the chip holds at once; workgroup b
// takes slots b, b + grid, b + 2 grid, ... (round-robin over the cost-sorted
// queue balances the load without atomics).
template <typename TIn, typename TOut, typename TS, typename TC, bool PERSIST>
__global__ __launch_bounds__(kThreads) void fov_fwd_kernel(const FwdLaunch a, const int32_t* __restrict__ radius,
                                                           const TC* __restrict__ wts,
                                                           const int32_t* __restrict__ order,
                                                           const FrameDesc* __restrict__ table,
                                                           const int32_t* __restrict__ prefix) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nslots = a.hdr ? a.hdr[2] : a.nslots;
    const int nframes = a.hdr ? a.hdr[0] : a.nframes;
    const int L = a.split_log2;
    for (int q = blockIdx.x; q < nslots; q += gridDim.x) {
        const int2 ent = reinterpret_cast<const int2*>(order)[q];  // (work item, radius word)
        int item = ent.x;
        if (item < 0) {  // empty slot
            if (!PERSIST) break;
            continue;
        }
        int c_lo = 0, c_hi = 1 << 30;  // channels of this item (clipped to the frame's below)
        if (a.cs_rmax >= 0 && (item & kChanItem)) {  // one channel of a fragment split by channel
            c_lo = (item >> kChanShift) & 15;
            c_hi = c_lo + 1;
            item &= kChanItemMask;
        }
        const int gid = item >> (2 * L);
        const int rr = ent.y;
        const int r = rr & 0xFFFF;
        Frag F = describe(table, prefix, nframes, gid);
        if (rr >> 16) {  // merged with the fragment below (same taps): one taller tile
            const Frag F2 = describe_at(F.fd, gid - F.lb, gid + F.fd->p.nbx);
            F.bh = F2.ya + F2.bh - F.ya;
        }
        if (!narrow_to_tile(F, L, item & ((1 << (2 * L)) - 1))) {
            if (!PERSIST) break;
            continue;
        }
        c_hi = min(c_hi, F.fd->c);
        if (c_lo < c_hi) process_fragment<TIn, TOut, TS, TC>(a, gid, r, F, c_lo, c_hi, wts, smem);
        if (!PERSIST) break;
        __syncthreads();  // this fragment's LDS reads are done before the next one is staged
    }
}

constexpr int kOrderThreads = 1024;
constexpr int kOrderMaxRings = 1024;
constexpr int kOrderCells = 12288;
constexpr int kOrderHeld = 4096;  // items whose (key, radius word) the order kernel holds in LDS
constexpr int kOrderBins = 16;  // angle bins per ring: one 16-lane segment of a wave scans a ring
constexpr int kXcds = 8;

// Rings (distinct radii) and angle bins of the order histogram.
int order_rings(int r_cap) { return std::min(r_cap + 1, kOrderMaxRings); }
int order_angle_bins(int nrings) { return std::max(1, std::min(kOrderBins, kOrderCells / nrings)); }

__device__ __forceinline__ int angle_bin(const Frag& F, int nang) {
    const FrameParams& fp = F.fd->p;
    const float half = 0.5f * (float)(fp.block - 1);
    const float cx = (float)(fp.origin_x + F.bx * fp.block) + half;
    const float cy = (float)(fp.origin_y + F.by * fp.block) + half;
    const float th = atan2f(cy - (float)fp.fix_y, cx - (float)fp.fix_x);  // (-pi, pi]
    int b = (int)((th + 3.14159265f) * (float)nang * 0.159154943f);
    return b < 0 ? 0 : (b >= nang ? nang - 1 : b);
}

// ---- plan kernels --------------------------------------------------------------------------------
// Fragment plan: radius and normalised taps, one wavefront per fragment.
template <typename TC>
__global__ __launch_bounds__(64) void fov_plan_weights_kernel(const FwdLaunch a, int32_t* __restrict__ radius,
                                                              int32_t* __restrict__ okey, int nrings, int nang,
                                                              TC* __restrict__ wts) {
    const int lane = threadIdx.x;
    const int nframes = a.hdr ? a.hdr[0] : a.nframes;
    const int nfrag = a.hdr ? a.hdr[1] : a.nfrag;
    for (int gid = blockIdx.x; gid < nfrag; gid += gridDim.x) {
    Frag F;
    if (a.from_args) {
        int f = 0;
        while (f + 1 < nframes && gid >= a.kprefix[f + 1]) ++f;
        F = describe_at(&a.fr[f], a.kprefix[f], gid);
        if (gid == 0) {
            // publish the frame table for the main kernel
            constexpr int kWords = sizeof(FrameDesc) / 4;
            const int32_t* src = reinterpret_cast<const int32_t*>(a.fr);
            int32_t* dst = reinterpret_cast<int32_t*>(a.table);
            for (int i = lane; i < nframes * kWords; i += 64) dst[i] = src[i];
            for (int i = lane; i <= nframes; i += 64) a.prefix[i] = a.kprefix[i];
        }
    } else {
        F = describe(a.table, a.prefix, nframes, gid);
    }
    const FrameParams& fp = F.fd->p;
    const double sigma = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[F.lb], fp.cap)
                                      : fragment_sigma_ramp(fp, F.bx, F.by);
    int r = radius_of(sigma);
    if (r > a.r_cap) r = a.r_cap;  // the host sized everything for r_cap; plans agree bit for bit
    // Vertical pairs at the cap (rows 2k and 2k+1, both sigma == cap, hence equal taps): the upper
    // fragment's item covers both, the lower one gets no item.
    int pair = 0;  // 1: upper of a merged pair, -1: lower
    if (a.merge && r > 0 && sigma == fp.cap) {
        const int by2 = F.by ^ 1;
        if (by2 < F.fd->nby) {
            const double s2 = fp.sigma_map ? clip_map_sigma((double)fp.sigma_map[F.lb + (by2 - F.by) * fp.nbx], fp.cap)
                                           : fragment_sigma_ramp(fp, F.bx, by2);
            if (s2 == fp.cap) pair = (F.by & 1) ? -1 : 1;
        }
    }
    if (lane == 0) {
        radius[gid] = r | (pair == 1 ? 0x10000 : 0);
        okey[gid] = pair == -1 ? -1  // no queue slot
                               : (nrings - 1 - min(r, nrings - 1)) * nang + angle_bin(F, nang);  // (ring, angle bin)
    }
    const int N = 2 * r + 1;
    const double inv = r > 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
    constexpr int kHeld = 4;  // taps per lane kept in registers
    double gv[kHeld];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kHeld; ++q) {
        const int j = lane + 64 * q;
        const double k = (double)(j - r);
        gv[q] = j < N ? exp(-(k * k) * inv) : 0.0;
        part += gv[q];
    }
    for (int j = lane + 64 * kHeld; j < N; j += 64) {
        const double k = (double)(j - r);
        part += exp(-(k * k) * inv);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    TC* wr = wts + (size_t)gid * a.wstride;
#pragma unroll
    for (int q = 0; q < kHeld; ++q) {
        const int j = lane + 64 * q;
        if (j < a.wstride) wr[j] = (TC)(gv[q] / part);
    }
    for (int j = lane + 64 * kHeld; j < a.wstride; j += 64) {
        double v = 0.0;
        if (j < N) {
            const double k = (double)(j - r);
            v = exp(-(k * k) * inv) / part;
        }
        wr[j] = (TC)v;
    }
    }
}

// Queue order.  Work items go by decreasing radius (their cost grows with r),
// so the costliest start first and the launch does not end on a long tail.
// The items of a split fragment share its (ring, angle bin) cell.
// Workgroup q runs on XCD q mod 8 (the dispatcher deals workgroups to the
// eight XCDs in turn), and each XCD has its own L2: neighbouring fragments
// share halo rows, so within every radius ring the fragments are sorted by
// angle around their frame's fixation and cut into eight contiguous arcs, arc
// a going to slots congruent to a mod 8.  Each XCD thus works through one
// angular sector ring by ring, with an equal share of every ring.  Rings are
// padded to a multiple of 8 slots with empty slots (-1).  With per-channel
// items (cs_rmax >= 0) the rings of radius <= cs_rmax follow the rest of the
// queue, each of their fragments in cmax consecutive slots of its arc's XCD
// (one per channel).
// One workgroup: LDS histogram over (ring, angle bin), scans, scatter; the
// order inside one (ring, angle bin) cell is arbitrary and results do not
// depend on it.  Up to kOrderHeld items keep their key and radius word in LDS
// from the histogram pass to the scatter, so memory is read once.

__global__ __launch_bounds__(kOrderThreads) void fov_order_kernel(const int32_t* __restrict__ okey,
                                                                  const int32_t* __restrict__ radius, int n_arg,
                                                                  int L, int nrings, int nang, int nslots_arg,
                                                                  const int32_t* __restrict__ hdr,
                                                                  int32_t* __restrict__ order, int cs_rmax,
                                                                  int cmax) {
    const int n = (hdr ? hdr[1] : n_arg) << (2 * L);  // work items
    const int nslots = hdr ? hdr[2] : nslots_arg;
    __shared__ int cells[kOrderCells];        // [ring][angle bin], ring 0 = largest radius
    __shared__ int ring_n[kOrderMaxRings];    // fragments per ring
    __shared__ int ring_base[kOrderMaxRings]; // first slot of each ring (multiple of 8)
    __shared__ int chan_base[kOrderMaxRings]; // split rings: first slot of each after the queue
    __shared__ int total_slots, total_extra;
    __shared__ int2 held[kOrderHeld];         // (key, radius word) per item when n <= kOrderHeld
    // rings whose fragments (r <= cs_rmax) are split by channel: ring >= small0
    const int small0 = (cs_rmax >= 0 && cmax > 1) ? max(nrings - 1 - cs_rmax, 0) : nrings;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ncell = nrings * nang;
    for (int i = tid; i < ncell; i += kOrderThreads) cells[i] = 0;
    __syncthreads();
    const bool hold = n <= kOrderHeld;
    for (int i = tid; i < n; i += kOrderThreads) {
        const int key = okey[i >> (2 * L)];
        if (hold) held[i] = make_int2(key, radius[i >> (2 * L)]);
        if (key >= 0) atomicAdd(&cells[key], 1);  // -1: the lower fragment of a merged pair
    }
    __syncthreads();
    // exclusive scan of the angle bins inside each ring: 16-lane segments, four rings per wave
    // (nang <= kOrderBins)
    for (int ring = wave * 4 + (lane >> 4); ring < nrings; ring += kOrderThreads / 16) {
        const int b = lane & 15;
        const bool live = ring < nrings && b < nang;
        const int v = live ? cells[ring * nang + b] : 0;
        int incl = v;
        for (int off = 1; off < 16; off <<= 1) {
            const int t = __shfl_up(incl, off, 16);
            if (b >= off) incl += t;
        }
        if (live) cells[ring * nang + b] = incl - v;
        if (ring < nrings && b == 15) ring_n[ring] = incl;
    }
    __syncthreads();
    if (wave == 0) {
        // ring bases: each ring takes 8 * ceil(n_ring / 8) slots (split rings go after the queue)
        int carry = 0;
        for (int r0 = 0; r0 < nrings; r0 += 64) {
            const int ring = r0 + lane;
            const int v = ring < small0 ? round_up(ring_n[ring], kXcds) : 0;
            int incl = v;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, 64);
                if (lane >= off) incl += t;
            }
            if (ring < nrings) ring_base[ring] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) total_slots = carry;
    } else if (wave == 1) {
        // split rings after the queue, ring by ring: cmax slots per fragment
        int carry = 0;
        for (int r0 = small0; r0 < nrings; r0 += 64) {
            const int ring = r0 + lane;
            const int v = ring < nrings ? round_up(ring_n[ring], kXcds) * cmax : 0;
            int incl = v;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, 64);
                if (lane >= off) incl += t;
            }
            if (ring < nrings) chan_base[ring] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) total_extra = carry;
    }
    __syncthreads();
    int2* ord = reinterpret_cast<int2*>(order);
    for (int i = tid; i < n; i += kOrderThreads) {
        const int2 kr = hold ? held[i] : make_int2(okey[i >> (2 * L)], radius[i >> (2 * L)]);
        const int key = kr.x;
        if (key < 0) continue;
        const int rr = kr.y;
        const int ring = key / nang;
        const int j = atomicAdd(&cells[key], 1);  // rank in the ring
        const int m = ring_n[ring];
        const int arc = (j * kXcds) / m;                  // arc a holds ranks [ceil(a m/8), ceil((a+1) m/8))
        const int k = j - (arc * m + kXcds - 1) / kXcds;  // rank inside the arc
        if (ring < small0) {
            ord[ring_base[ring] + kXcds * k + arc] = make_int2(i, rr);
        } else {  // one slot per channel, consecutive slots of the same XCD
            const int e = total_slots + chan_base[ring] + kXcds * k * cmax + arc;
            for (int ch = 0; ch < cmax; ++ch) ord[e + kXcds * ch] = make_int2(i | kChanItem | (ch << kChanShift), rr);
        }
    }
    // empty slots: arc a of a ring of m holds ceil((a+1)m/8) - ceil(a m/8) fragments, ceil(m/8)
    // or one fewer, so each arc leaves at most its last slot empty (eight lanes per ring)
    for (int ring = tid >> 3; ring < nrings; ring += kOrderThreads / kXcds) {
        const int arc = tid & (kXcds - 1);
        const int m = ring_n[ring], per = (m + kXcds - 1) / kXcds;
        const int sz = ((arc + 1) * m + kXcds - 1) / kXcds - (arc * m + kXcds - 1) / kXcds;
        if (sz == per) continue;
        const int k = per - 1;
        if (ring < small0) {
            ord[ring_base[ring] + kXcds * k + arc] = make_int2(-1, 0);
        } else {
            const int e = total_slots + chan_base[ring] + kXcds * k * cmax + arc;
            for (int ch = 0; ch < cmax; ++ch) ord[e + kXcds * ch] = make_int2(-1, 0);
        }
    }
    for (int q = total_slots + total_extra + tid; q < nslots; q += kOrderThreads) ord[q] = make_int2(-1, 0);
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

template <typename TIn, typename TOut, typename TS, typename TC, bool PERSIST>
fov_status launch_main(const FwdLaunch& a, size_t lds, const PlanBuffers& plan, hipStream_t stream,
                       size_t lds_limit, int cus, hipEvent_t ev_start, hipEvent_t ev_stop) {
    auto kern = fov_fwd_kernel<TIn, TOut, TS, TC, PERSIST>;
    fov_status st = allow_dyn_lds((const void*)kern, lds_limit);
    if (st != FOV_OK) return st;
    int grid = a.nslots;
    if (PERSIST) grid = std::max(1, std::min(a.nslots, std::max(occupancy_of((const void*)kern, lds), 1) * cus));
    if (ev_start || ev_stop) {
        // The dispatch itself stamps the events: no separate event packets (each would leave a
        // gap of several microseconds between the kernels of the stream).
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, stream, ev_start, ev_stop, 0, a,
                              (const int32_t*)plan.radius, (const TC*)plan.weights, (const int32_t*)plan.order,
                              (const FrameDesc*)a.table, (const int32_t*)a.prefix);
    } else {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, stream, a, (const int32_t*)plan.radius,
                           (const TC*)plan.weights, (const int32_t*)plan.order, (const FrameDesc*)a.table,
                           (const int32_t*)a.prefix);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "forward kernel launch");
    return FOV_OK;
}

template <typename TIn, typename TOut, typename TS, typename TC>
fov_status launch_typed(const FwdLaunch& a, size_t lds, const PlanBuffers& plan, hipStream_t stream,
                        size_t lds_limit, int cus, bool persist, hipEvent_t ev_start, hipEvent_t ev_stop) {
    TC* wts = static_cast<TC*>(plan.weights);
    const int nrings = order_rings(a.r_cap), nang = order_angle_bins(nrings);
    const int plan_grid = a.hdr ? std::min(a.nfrag, 8192) : a.nfrag;
    hipLaunchKernelGGL(fov_plan_weights_kernel<TC>, dim3(plan_grid), dim3(64), 0, stream, a, plan.radius, plan.okey,
                       nrings, nang, wts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "plan kernel launch");
    hipLaunchKernelGGL(fov_order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, (const int32_t*)plan.okey,
                       (const int32_t*)plan.radius, a.nfrag,
                       a.split_log2, nrings, nang, a.nslots, a.hdr, plan.order, a.cs_rmax, a.cmax);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "order kernel launch");
    if (persist) return launch_main<TIn, TOut, TS, TC, true>(a, lds, plan, stream, lds_limit, cus, ev_start, ev_stop);
    return launch_main<TIn, TOut, TS, TC, false>(a, lds, plan, stream, lds_limit, cus, ev_start, ev_stop);
}

int stage_size(int in_dtype) { return in_dtype == FOV_U8 ? 2 : (in_dtype == FOV_F32 ? 4 : 8); }
int compute_size(int in_dtype) { return in_dtype == FOV_F64 ? 8 : 4; }

}  // namespace

int queue_slots(int nitems, int r_cap) { return nitems + kXcds * order_rings(r_cap); }

int queue_slots_by_channel(int nfrag, int r_cap, int cmax) { return cmax * queue_slots(nfrag, r_cap); }

size_t plan_bytes(int nfrag, int nslots, int wstride, int wsize) {
    return 2 * align16((size_t)nfrag * 4) + align16((size_t)nslots * 8) + 256 + (size_t)nfrag * wstride * wsize;
}

PlanBuffers carve_plan(void* ws, int nfrag, int nslots) {
    PlanBuffers p;
    char* base = static_cast<char*>(ws);
    const size_t f4 = align16((size_t)nfrag * 4);
    p.radius = reinterpret_cast<int32_t*>(base);
    p.okey = reinterpret_cast<int32_t*>(base + f4);
    p.order = reinterpret_cast<int32_t*>(base + 2 * f4);
    p.weights = base + 2 * f4 + align16((size_t)nslots * 8) + 256;
    return p;
}

int forward_strip_max() { return kStripMax; }

int forward_tile_rows(int r, int tile_h) { return geom(r, 1, tile_h).TH; }

size_t forward_lds_bytes(int in_dtype, int r_cap, int tile_w, int tile_h, int strip_rows) {
    const Geom g = geom(r_cap, tile_w, tile_h);
    int rows = strip_rows < g.TH ? strip_rows : g.TH;
    if (rows > kStripMax) rows = kStripMax;
    const int es = stage_size(in_dtype), ec = compute_size(in_dtype);
    // 8-bit input: (-r) mod 4 leading columns; 2r + ((-r) mod 4) never decreases with r, so r_cap sizes them
    const int TW = g.TW + (in_dtype == FOV_U8 ? ((-r_cap) & 3) : 0);
    return kTileLead + tap_lds_bytes(r_cap, ec) + align16((size_t)rows * tile_pitch(TW, es) * es) +
           (size_t)g.G * kPH * inter_pitch(g.TH, ec) * ec + 64;
}

fov_status launch_forward(const FwdLaunch& a, int in_dtype, int out_dtype, size_t lds, const PlanBuffers& plan,
                          hipStream_t stream, size_t lds_limit, int cus, bool persist, hipEvent_t ev_start,
                          hipEvent_t ev_stop) {
    if (a.nfrag <= 0) return FOV_OK;
    if (in_dtype == FOV_U8 && out_dtype == FOV_U8)
        return launch_typed<uint8_t, uint8_t, _Float16, float>(a, lds, plan, stream, lds_limit, cus, persist, ev_start, ev_stop);
    if (in_dtype == FOV_U8 && out_dtype == FOV_F32)
        return launch_typed<uint8_t, float, _Float16, float>(a, lds, plan, stream, lds_limit, cus, persist, ev_start, ev_stop);
    if (in_dtype == FOV_F32 && out_dtype == FOV_F32)
        return launch_typed<float, float, float, float>(a, lds, plan, stream, lds_limit, cus, persist, ev_start, ev_stop);
    if (in_dtype == FOV_F64 && out_dtype == FOV_F64)
        return launch_typed<double, double, double, double>(a, lds, plan, stream, lds_limit, cus, persist, ev_start, ev_stop);
    return set_error(FOV_EDTYPE, "unsupported dtype pair");
}

int forward_occupancy(int in_dtype, int out_dtype, size_t lds) {
    const void* k = forward_main_kernel(in_dtype, out_dtype, false);
    return k ? occupancy_of(k, lds) : 0;
}

const void* forward_main_kernel(int in_dtype, int out_dtype, bool persist) {
    if (in_dtype == FOV_U8 && out_dtype == FOV_U8)
        return persist ? (const void*)fov_fwd_kernel<uint8_t, uint8_t, _Float16, float, true>
                       : (const void*)fov_fwd_kernel<uint8_t, uint8_t, _Float16, float, false>;
    if (in_dtype == FOV_U8 && out_dtype == FOV_F32)
        return persist ? (const void*)fov_fwd_kernel<uint8_t, float, _Float16, float, true>
                       : (const void*)fov_fwd_kernel<uint8_t, float, _Float16, float, false>;
    if (in_dtype == FOV_F32 && out_dtype == FOV_F32)
        return persist ? (const void*)fov_fwd_kernel<float, float, float, float, true>
                       : (const void*)fov_fwd_kernel<float, float, float, float, false>;
    if (in_dtype == FOV_F64 && out_dtype == FOV_F64)
        return persist ? (const void*)fov_fwd_kernel<double, double, double, double, true>
                       : (const void*)fov_fwd_kernel<double, double, double, double, false>;
    return nullptr;
}

fov_status launch_plan(const FrameParams& fp, int nblk, double* sigma_out, int32_t* r_out, hipStream_t stream) {
    if (nblk <= 0) return FOV_OK;
    hipLaunchKernelGGL(fov_plan_kernel, dim3((nblk + 255) / 256), dim3(256), 0, stream, fp, nblk, sigma_out, r_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "plan kernel launch");
    return FOV_OK;
}

}  // namespace fov
