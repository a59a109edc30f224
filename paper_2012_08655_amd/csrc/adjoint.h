// Launch interface of the adjoint (backward) kernels.
#pragma once

#include "common.h"
#include "forward.h"

namespace fov {

// Shape constants of one adjoint launch (frames, plan and frame table travel
// as for the forward, in a FwdLaunch).
struct AdjShape {
    int32_t bmax;     // largest fragment side
    int32_t sw;       // columns of a transposed window in scratch: bmax + 2 r_cap
    int32_t sh;       // column stride of a window in scratch (a multiple of 128 bytes)
    int32_t cmax;     // largest channel count
    int32_t pitch_a;  // LDS row pitch of the vertical transpose's rows (zero columns around the data)
    int32_t pad_b;    // zero rows above a staged gradient column
    int32_t pitch_b;  // LDS column pitch of the staged gradient
    int32_t rows_r;   // window rows the window kernel transposes per run (a multiple of 4)
    int32_t tap_stride;  // LDS elements per copy of the taps (a multiple of 4)
    int32_t tap_elems;   // LDS elements of the tap copies (16 / element size copies)
    uint32_t bdiv;       // ceil(2^32 / bmax) (0 for bmax = 1): i / bmax = mulhi(i, bdiv) for i * bmax < 2^32
};

// LDS the window kernel aims to stay within (the window's rows are transposed in runs beyond it).
constexpr size_t kAdjLdsBudget = (size_t)96 << 10;

// Leading zero taps before each copy of a fragment's taps in LDS: windows may
// start up to three taps early (to keep 16-byte LDS loads aligned) and read
// zeros there.
constexpr int kAdjWeightLead = 4;

// Rows before a fragment's first row in its window columns: r rounded up to
// 128 bytes of elements of size es.
__host__ __device__ inline int window_lead(int r, int es) { return round_up(r, 128 / es); }

AdjShape adjoint_shape(int es, int r_cap, int bmax, int cmax);
// Dynamic LDS of the window kernel.
size_t adjoint_lds(const AdjShape& s, int es);
// Scratch elements for nfrag fragments.
size_t adjoint_scratch_elems(const AdjShape& s, int nfrag);

// Window and sum kernels for the fragments of `a`: each fragment's radius
// (into radius[], one entry per fragment), taps and transposed window into
// scratch, then every output tile as the sum of the windows that reach it.
// es = 4 (float) or 8 (double).
fov_status launch_adjoint(const FwdLaunch& a, const AdjShape& s, int es, int32_t* radius, void* scratch,
                          hipStream_t stream, size_t lds_limit);

}  // namespace fov
