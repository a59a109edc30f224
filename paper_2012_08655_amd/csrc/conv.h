// Device building blocks shared by the forward and adjoint kernels: LDS
// pitches, the register-window 1-D correlations of the horizontal and
// vertical passes, and fragment lookup in a launch's frame table.
#pragma once

#include <hip/hip_runtime.h>

#include "forward.h"

namespace fov {
namespace {

constexpr int kPH = 8;  // outputs per thread, horizontal pass
constexpr int kPV = 4;  // outputs per thread, vertical pass
constexpr int kU = 4;   // taps per register-window step

// Window loads run up to 3 elements past the last staged column and 4 rows
// past the last intermediate row (values that no tap uses); the pitch and the
// allocation leave room for them.
constexpr int kColSlack = 4;
constexpr int kRowSlack = 4;

// Tile row pitch in elements.  A horizontal-pass lane reads 4 elements (4*es
// bytes) per load from its own row, and the lanes of a group sit on
// consecutive rows; rows start 4*es bytes apart modulo 128 so that 128/(4*es)
// such lanes cover the 32 LDS banks once.
__host__ __device__ inline int tile_pitch(int TW, int es) {
    const int q = 4, m = 128 / es;
    const int need = TW + kColSlack;
    return round_up(need > q ? need - q : 1, m) + q;
}

// The intermediate is stored column-major (one column of TH rows after
// another) so the vertical pass reads four rows with one 16-byte load.  Column
// pitch in elements: columns start 16 bytes apart modulo 128 bytes (eight
// lanes on eight consecutive columns hit 32 distinct banks), with room for
// the window's overrun past the last row.
__host__ __device__ inline int inter_pitch(int TH, int es) {
    const int q = 16 / es, m = 128 / es;
    const int need = TH + kRowSlack;
    return round_up(need > q ? need - q : 1, m) + q;
}

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS bytes of a forward workgroup's taps for radii up to r_cap: all 2r+1 taps (for the vertical
// and the plain horizontal pass), then w_1 .. w_r again from a 16-byte boundary (for the
// symmetric pass), each list padded to whole 4-tap groups.
__host__ __device__ inline size_t tap_lds_bytes(int r_cap, int ec) {
    return align16((size_t)(round_up(2 * r_cap + 1, 4) + round_up(r_cap, 4) + 4) * ec);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Smallest s with 2^s >= v (v >= 1).
__host__ __device__ inline int ceil_log2(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

// Frame buffers as global-memory pointers (pointers read from the frame table would otherwise be
// accessed with flat instructions).
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(T* p) {
    return (global_ptr<T>)p;
}

// Index of the calling wavefront in its workgroup, as a scalar (uniform) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

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

// Horizontal step: taps j0..j0+NT-1 on 8 outputs; window = X ++ Y ++ Z[0..2].
template <int NT = kU, typename TC, typename TS>
__device__ __forceinline__ void hstep(TC (&acc)[kPH], const TS (&X)[4], const TS (&Y)[4], const TS (&Z)[4],
                                      const TC* __restrict__ w) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const TC wu = w[u];
#pragma unroll
        for (int p = 0; p < kPH; ++p) {
            const int i = p + u;
            const TS v = i < 4 ? X[i] : (i < 8 ? Y[i - 4] : Z[i - 8]);
            acc[p] = fma(wu, (TC)v, acc[p]);
        }
    }
}

// Vertical step: taps j0..j0+NT-1 on 4 outputs; window = X ++ Y[0..2].
template <int NT = kU, typename TC>
__device__ __forceinline__ void vstep(TC (&acc)[kPV], const TC (&X)[4], const TC (&Y)[4], const TC* __restrict__ w) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const TC wu = w[u];
#pragma unroll
        for (int p = 0; p < kPV; ++p) {
            const int i = p + u;
            acc[p] = fma(wu, i < 4 ? X[i] : Y[i - 4], acc[p]);
        }
    }
}

// Partial horizontal step of nt (1..3) taps.
template <typename TC, typename TS>
__device__ __forceinline__ void hstep_part(int nt, TC (&acc)[kPH], const TS (&X)[4], const TS (&Y)[4],
                                           const TS (&Z)[4], const TC* __restrict__ w) {
    if (nt == 1) hstep<1>(acc, X, Y, Z, w);
    else if (nt == 2) hstep<2>(acc, X, Y, Z, w);
    else hstep<3>(acc, X, Y, Z, w);
}

// 8 horizontal outputs from a staged row: N taps over inputs row[0 .. N+6].
// Three 4-value buffers rotate through a 3-step unrolled loop, so no window
// value is ever moved between registers.
template <typename TC, typename TS>
__device__ __forceinline__ void hconv(TC (&acc)[kPH], const TS* row, int N, const TC* __restrict__ w) {
    TS A[4], B[4], C[4];
    load4_row(row, A);
    load4_row(row + 4, B);
    int j0 = 0;
    for (; j0 + 12 <= N; j0 += 12) {
        load4_row(row + j0 + 8, C);
        hstep(acc, A, B, C, w + j0);
        load4_row(row + j0 + 12, A);
        hstep(acc, B, C, A, w + j0 + 4);
        load4_row(row + j0 + 16, B);
        hstep(acc, C, A, B, w + j0 + 8);
    }
    int left = N - j0;  // 0..11, window state (A, B)
    if (left == 0) return;
    load4_row(row + j0 + 8, C);
    if (left < 4) { hstep_part(left, acc, A, B, C, w + j0); return; }
    hstep(acc, A, B, C, w + j0);
    j0 += 4; left -= 4;  // state (B, C)
    if (left == 0) return;
    load4_row(row + j0 + 8, A);
    if (left < 4) { hstep_part(left, acc, B, C, A, w + j0); return; }
    hstep(acc, B, C, A, w + j0);
    j0 += 4; left -= 4;  // state (C, A), left 0..3
    if (left == 0) return;
    load4_row(row + j0 + 8, B);
    hstep_part(left, acc, C, A, B, w + j0);
}

// ---- symmetric horizontal pass for 8-bit input staged as 16-bit integers ----------------------
// The taps are symmetric (w_{-k} = w_k), so out[p] = w_0 x[p] + sum_k w_k (x[p-k] + x[p+k]).  The
// staged values are integers 0..255, two per 32-bit register, so one 32-bit integer add forms two
// such pair sums exactly (at most 510: no carry crosses into the upper half), and one
// v_fma_mix_f32 per output and distance multiplies a sum by the FP32 weight.  The mixed FMA reads
// a 16-bit sum s as the fp16 subnormal s * 2^-24, and the weights it gets are scaled by 2^24
// (kSymScale), so it forms the exact product w_k * s as with an unscaled weight and an fp16 s.
// 4.5 adds and 8 FMAs per distance for 8 outputs instead of 16 FMAs; the integer add is a VALU
// form that the hardware can issue beside another wave's instruction in the same cycle.  Two
// samples of a 32-bit register are the outputs (2q, 2q+1) at even distances and (2q-1, 2q) at odd
// ones; with the centre of output 0 on a 4-sample boundary every operand is a whole register.  At
// odd distances the outer registers use one half only: the lower halves there are staged samples
// (the tile starts (-r) mod 4 columns left of the padded tile, so the sample left of output 0's
// window at an odd r is staged), and whatever the upper half of the last one holds, a carry out
// of it is dropped.
constexpr float kSymScale = 16777216.0f;  // 2^24
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2v as_h2(uint32_t u) { return __builtin_bit_cast(h2v, u); }

__device__ __forceinline__ uint2 load_grp(const _Float16* p) { return *reinterpret_cast<const uint2*>(p); }

// Distance k: l[q] holds samples (p-k, p+1-k) and t[q] samples (p+k, p+1+k) of the output pair
// starting at p = 2q (even k) or p = 2q-1 (odd k).
template <bool ODD>
__device__ __forceinline__ void sym_tap(float (&acc)[kPH], const uint32_t* l, const uint32_t* t, float wk) {
    if constexpr (ODD) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const h2v s = as_h2(l[q] + t[q]);
            if (q > 0) acc[2 * q - 1] = fmaf(wk, (float)s.x, acc[2 * q - 1]);
            if (q < 4) acc[2 * q] = fmaf(wk, (float)s.y, acc[2 * q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const h2v s = as_h2(l[q] + t[q]);
            acc[2 * q] = fmaf(wk, (float)s.x, acc[2 * q]);
            acc[2 * q + 1] = fmaf(wk, (float)s.y, acc[2 * q + 1]);
        }
    }
}

// Distances 4m+1 .. 4m+NT.  Left groups L0 < L1 < L2 hold samples c-4m-4 .. c-4m+7 and right
// groups R0 < R1 < R2 samples c+4m .. c+4m+11 (c: centre of output 0).
template <int NT>
__device__ __forceinline__ void sym_block(float (&acc)[kPH], uint2 L0, uint2 L1, uint2 L2, uint2 R0, uint2 R1,
                                          uint2 R2, const float* __restrict__ wk) {
    const uint32_t l[6] = {L0.x, L0.y, L1.x, L1.y, L2.x, L2.y};
    const uint32_t t[6] = {R0.x, R0.y, R1.x, R1.y, R2.x, R2.y};
    if (NT >= 1) sym_tap<true>(acc, l + 1, t, wk[0]);
    if (NT >= 2) sym_tap<false>(acc, l + 1, t + 1, wk[1]);
    if (NT >= 3) sym_tap<true>(acc, l, t + 1, wk[2]);
    if (NT >= 4) sym_tap<false>(acc, l, t + 2, wk[3]);
}

__device__ __forceinline__ void sym_part(int nt, float (&acc)[kPH], uint2 L0, uint2 L1, uint2 L2, uint2 R0, uint2 R1,
                                         uint2 R2, const float* __restrict__ wk) {
    if (nt == 1) sym_block<1>(acc, L0, L1, L2, R0, R1, R2, wk);
    else if (nt == 2) sym_block<2>(acc, L0, L1, L2, R0, R1, R2, wk);
    else sym_block<3>(acc, L0, L1, L2, R0, R1, R2, wk);
}

// 8 horizontal outputs, radius r >= 1.  rc points at the centre of output 0 (8-byte aligned);
// w0 = 2^24 w_0 and ws[j] = 2^24 w_{j+1} for j = 0..r-1 (16-byte aligned).  Reads samples rc[-r-3 .. r+10]:
// the ones outside [-r, r+7] fall in halves whose sums no output uses.  Sums are taken in the
// order k = 0, 1, .., r.
__device__ __forceinline__ void hconv_sym(float (&acc)[kPH], const _Float16* rc, int r, float w0,
                                          const float* __restrict__ ws) {
    uint2 LA = load_grp(rc), LB = load_grp(rc + 4), LC;
    uint2 RA = LA, RB = LB, RC;
    {
        const uint32_t x[4] = {LA.x, LA.y, LB.x, LB.y};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[2 * q] = fmaf(w0, (float)as_h2(x[q]).x, acc[2 * q]);
            acc[2 * q + 1] = fmaf(w0, (float)as_h2(x[q]).y, acc[2 * q + 1]);
        }
    }
    // Three buffers per side rotate through a 3-block unrolled loop: block m loads the left group
    // at c-4m-4 and the right group at c+4m+8 into the buffers the previous block released.
    const int M = r >> 2, NT = r & 3;
    int m = 0;
    for (; m + 3 <= M; m += 3) {
        LC = load_grp(rc - 4 * (m + 1));
        RC = load_grp(rc + 4 * (m + 2));
        sym_block<4>(acc, LC, LA, LB, RA, RB, RC, ws + 4 * m);
        LB = load_grp(rc - 4 * (m + 2));
        RA = load_grp(rc + 4 * (m + 3));
        sym_block<4>(acc, LB, LC, LA, RB, RC, RA, ws + 4 * m + 4);
        LA = load_grp(rc - 4 * (m + 3));
        RB = load_grp(rc + 4 * (m + 4));
        sym_block<4>(acc, LA, LB, LC, RC, RA, RB, ws + 4 * m + 8);
    }
    if (m == M && NT == 0) return;
    LC = load_grp(rc - 4 * (m + 1));
    RC = load_grp(rc + 4 * (m + 2));
    if (m == M) { sym_part(NT, acc, LC, LA, LB, RA, RB, RC, ws + 4 * m); return; }
    sym_block<4>(acc, LC, LA, LB, RA, RB, RC, ws + 4 * m);
    ++m;
    if (m == M && NT == 0) return;
    LB = load_grp(rc - 4 * (m + 1));
    RA = load_grp(rc + 4 * (m + 2));
    if (m == M) { sym_part(NT, acc, LB, LC, LA, RB, RC, RA, ws + 4 * m); return; }
    sym_block<4>(acc, LB, LC, LA, RB, RC, RA, ws + 4 * m);
    ++m;
    if (NT == 0) return;  // m == M here
    LA = load_grp(rc - 4 * (m + 1));
    RB = load_grp(rc + 4 * (m + 2));
    sym_part(NT, acc, LA, LB, LC, RC, RA, RB, ws + 4 * m);
}

// 4 horizontal outputs, the same pass for strips of few rows: a 16-row block of 8-output tasks
// fills one wave, so a strip of one or two blocks would leave waves idle; with 4-output tasks
// twice as many lanes share it.  The pairs are outputs (0, 1), (2, 3) at even distances and
// (-1, 0), (1, 2), (3, 4) at odd ones, each output takes the same pair sums and FMAs in the same
// order as in hconv_sym (bitwise the same results), and its reads (rc[-r-3 .. r+6]) stay
// within those of the 8-output task whose columns it shares.
template <bool ODD>
__device__ __forceinline__ void sym_tap4(float (&acc)[4], const uint32_t* l, const uint32_t* t, float wk) {
    if constexpr (ODD) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const h2v s = as_h2(l[q] + t[q]);
            if (q > 0) acc[2 * q - 1] = fmaf(wk, (float)s.x, acc[2 * q - 1]);
            if (q < 2) acc[2 * q] = fmaf(wk, (float)s.y, acc[2 * q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const h2v s = as_h2(l[q] + t[q]);
            acc[2 * q] = fmaf(wk, (float)s.x, acc[2 * q]);
            acc[2 * q + 1] = fmaf(wk, (float)s.y, acc[2 * q + 1]);
        }
    }
}

// Distances 4m+1 .. 4m+NT: L0 < L1 hold samples c-4m-4 .. c-4m+3, R0 < R1 samples c+4m .. c+4m+7.
template <int NT>
__device__ __forceinline__ void sym_block4(float (&acc)[4], uint2 L0, uint2 L1, uint2 R0, uint2 R1,
                                           const float* __restrict__ wk) {
    const uint32_t l[4] = {L0.x, L0.y, L1.x, L1.y};
    const uint32_t t[4] = {R0.x, R0.y, R1.x, R1.y};
    if (NT >= 1) sym_tap4<true>(acc, l + 1, t, wk[0]);
    if (NT >= 2) sym_tap4<false>(acc, l + 1, t + 1, wk[1]);
    if (NT >= 3) sym_tap4<true>(acc, l, t + 1, wk[2]);
    if (NT >= 4) sym_tap4<false>(acc, l, t + 2, wk[3]);
}

// rc, w0 and ws as for hconv_sym.
__device__ __forceinline__ void hconv_sym4(float (&acc)[4], const _Float16* rc, int r, float w0,
                                           const float* __restrict__ ws) {
    uint2 Lc = load_grp(rc), Rc = Lc;  // the block's inner groups: c-4m and c+4m
    {
        const uint32_t x[2] = {Lc.x, Lc.y};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            acc[2 * q] = fmaf(w0, (float)as_h2(x[q]).x, acc[2 * q]);
            acc[2 * q + 1] = fmaf(w0, (float)as_h2(x[q]).y, acc[2 * q + 1]);
        }
    }
    const int M = r >> 2, NT = r & 3;
    for (int m = 0; m < M; ++m) {
        const uint2 L0 = load_grp(rc - 4 * (m + 1));
        const uint2 R1 = load_grp(rc + 4 * (m + 1));
        sym_block4<4>(acc, L0, Lc, Rc, R1, ws + 4 * m);
        Lc = L0;
        Rc = R1;
    }
    if (NT == 0) return;
    const uint2 L0 = load_grp(rc - 4 * (M + 1));
    const uint2 R1 = load_grp(rc + 4 * (M + 1));
    if (NT == 1) sym_block4<1>(acc, L0, Lc, Rc, R1, ws + 4 * M);
    else if (NT == 2) sym_block4<2>(acc, L0, Lc, Rc, R1, ws + 4 * M);
    else sym_block4<3>(acc, L0, Lc, Rc, R1, ws + 4 * M);
}

template <typename TC>
__device__ __forceinline__ void vstep_part(int nt, TC (&acc)[kPV], const TC (&X)[4], const TC (&Y)[4],
                                           const TC* __restrict__ w) {
    if (nt == 1) vstep<1>(acc, X, Y, w);
    else if (nt == 2) vstep<2>(acc, X, Y, w);
    else vstep<3>(acc, X, Y, w);
}

// 4 vertical outputs from a column of the (column-major) intermediate: N
// taps over col[0 .. N+2]; two buffers alternate through a 2-step loop.
template <typename TC>
__device__ __forceinline__ void vconv(TC (&acc)[kPV], const TC* col, int N, const TC* __restrict__ w) {
    TC A[4], B[4];
    load4_row(col, A);
    int j0 = 0;
    for (; j0 + 8 <= N; j0 += 8) {
        load4_row(col + j0 + 4, B);
        vstep(acc, A, B, w + j0);
        load4_row(col + j0 + 8, A);
        vstep(acc, B, A, w + j0 + 4);
    }
    int left = N - j0;  // 0..7, state A
    if (left == 0) return;
    load4_row(col + j0 + 4, B);
    if (left < 4) { vstep_part(left, acc, A, B, w + j0); return; }
    vstep(acc, A, B, w + j0);
    j0 += 4; left -= 4;  // state B
    if (left == 0) return;
    load4_row(col + j0 + 4, A);
    vstep_part(left, acc, B, A, w + j0);
}

// Division by a value d >= 1 fixed for a launch or work item: div_magic(d) = ceil(2^32 / d) (0 for
// d = 1), and x / d = div_by(x, div_magic(d)) for 0 <= x with x * d < 2^32 (the multiplier's excess
// over 2^32 / d is below 1, so it moves x / d by less than x * d / 2^32 < 1 of 1/d).
__host__ __device__ inline uint32_t div_magic(uint32_t d) { return d > 1 ? 0xFFFFFFFFu / d + 1u : 0u; }

__device__ __forceinline__ int div_by(int x, uint32_t m) { return m ? (int)__umulhi((uint32_t)x, m) : x; }

// ---- fragments of a launch ---------------------------------------------------------------------
// Last frame whose first fragment is <= gid (prefix has nframes+1 entries).
__device__ __forceinline__ int frame_search(const int32_t* __restrict__ prefix, int nframes, int gid) {
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= gid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Everything the kernels need to know about one fragment.
struct Frag {
    const FrameDesc* fd;
    int lb, bx, by, xa, ya, bw, bh;
};

__device__ __forceinline__ Frag describe_at(const FrameDesc* fd, int first, int gid) {
    Frag F;
    F.fd = fd;
    const FrameParams& fp = fd->p;
    F.lb = gid - first;
    F.by = F.lb / fp.nbx;
    F.bx = F.lb - F.by * fp.nbx;
    const int B = fp.block;
    const int X0 = fp.origin_x + F.bx * B, Y0 = fp.origin_y + F.by * B;
    F.xa = max(X0, 0);
    F.ya = max(Y0, 0);
    F.bw = min(X0 + B, fd->w) - F.xa;
    F.bh = min(Y0 + B, fd->h) - F.ya;
    return F;
}

// Fragment gid, reading frames from the device table (main kernel).
__device__ __forceinline__ Frag describe(const FrameDesc* __restrict__ table, const int32_t* __restrict__ prefix,
                                         int nframes, int gid) {
    const int f = frame_search(prefix, nframes, gid);
    return describe_at(table + f, prefix[f], gid);
}

}  // namespace
}  // namespace fov
