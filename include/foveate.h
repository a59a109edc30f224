/*
 * foveate.h -- C ABI of libfoveate.so, block-wise foveation on AMD MI355X
 * (gfx950).
 *
 * The method (Malkin, Deza, Poggio, arXiv 2012.08655): a frame is cut into
 * square fragments of side B; each fragment is blurred with one Gaussian whose
 * strength follows the distance from the fragment midpoint to the fixation
 * point (Sec. 2 "Block-wise Foveation", Fig. 1).  The Gaussian is Eq. (1)
 * sampled at integer offsets, cut off beyond 3 sigma and normalised to sum 1
 * (Appendix "Methods"); a foveal fragment is copied unchanged (Appendix
 * "Workload of the Block").  Blurring is separable: a horizontal pass into an
 * on-chip intermediate, then a vertical pass (Sec. 2, Alg. 1).
 *
 * Conventions used throughout:
 *   - Coordinates are pixel-centre: (0,0) is the centre of the top-left pixel;
 *     "image centre" of a w x h frame is ((w-1)/2, (h-1)/2).
 *   - Fragment (bx, by) covers x in [origin_x + bx*B, origin_x + (bx+1)*B) and
 *     y likewise, clipped to the frame; its midpoint is
 *     (origin_x + bx*B + (B-1)/2, origin_y + by*B + (B-1)/2), also for
 *     clipped edge fragments.
 *   - sigma(e) = 0 when e < e0, else min(slope*(e - e0), cap); radius
 *     r = ceil(3*sigma) in IEEE double; N = 2r+1 taps w_k = exp(-k^2/(2 sigma^2)),
 *     normalised; a fragment with sigma = 0 is copied.
 *   - Pixels beyond the frame edge take the value of the nearest edge pixel
 *     (clamp-to-edge, per axis).
 *   - u8 output: round half to even, clip to 0..255.  u8 input is convolved
 *     in float32 on the raw 0..255 scale.
 *
 * Memory: the caller owns every pixel buffer (device memory).  The library
 * never allocates or frees caller buffers.  forward/backward are asynchronous
 * and ordered on the caller's HIP stream; they return once work is enqueued.
 *
 * Errors: every call returns a fov_status; 0 is success.  Calls never throw
 * and never abort.  foveate_last_error() returns a thread-local description
 * of the last non-OK status.
 */
#ifndef FOVEATE_H
#define FOVEATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FOV_OK = 0,
    FOV_EINVAL = -1,    /* bad argument: null pointer, shape mismatch, bad parameter   */
    FOV_EDTYPE = -2,    /* unsupported dtype or dtype pair                             */
    FOV_ELAYOUT = -3,   /* negative strides or a self-overlapping output layout         */
    FOV_EALIAS = -4,    /* output memory overlaps input memory                         */
    FOV_ENOMEM = -5,    /* a library-internal device or pinned allocation failed       */
    FOV_EAGAIN = -6,    /* server request table full; retry after polling             */
    FOV_EHIP = -7,      /* a HIP runtime call failed; see foveate_last_error()         */
    FOV_ECLOSED = -8,   /* server is shutting down                                     */
    FOV_ENOTICKET = -9, /* unknown or already-retired ticket                           */
    FOV_ERANGE = -10    /* a fragment radius exceeds what on-chip memory can hold      */
} fov_status;

typedef enum { FOV_U8 = 0, FOV_F32 = 1, FOV_F64 = 2 } fov_dtype;

/*
 * A strided 4-D view of device memory, logical dims (n, c, h, w) with
 * element strides (not bytes).  HWC u8 frames and NCHW float tensors are both
 * described by choosing strides: an n x h x w x 3 u8 batch has
 * sn = h*w*3, sc = 1, sh = w*3, sw = 3.  Strides must be >= 0.
 */
typedef struct {
    void* data;        /* device pointer; may be NULL only if the view is empty */
    int32_t dtype;     /* fov_dtype */
    int32_t n, c, h, w;
    int64_t sn, sc, sh, sw;
} fov_tensor;

/* Per-frame foveation parameters (all distances in pixels). */
typedef struct {
    double fix_x, fix_y; /* fixation point, pixel-centre coordinates (finite)     */
    double e0;           /* foveal radius: fragments nearer than e0 are copied      */
    double slope;        /* sigma increase per px beyond e0 (>= 0)                  */
    double cap;          /* largest sigma (>= 0)                                    */
    int32_t block;       /* fragment side B, 1..64 (the paper's headline uses 32)   */
    int32_t origin_x;    /* left edge of fragment column 0, in (-B, 0]; 0 = plain   */
    int32_t origin_y;    /* top edge of fragment row 0, in (-B, 0]; 0 = plain       */
    int32_t reserved;    /* must be 0                                               */
    const float* sigma_map; /* optional device array [nby*nbx] (row-major) giving
                               each fragment's sigma directly, in place of the
                               ramp (Sec. 4: any image may define blur strength);
                               values are clipped to [0, cap]; NaN counts as 0.
                               NULL = use the ramp.                              */
} fov_params;

/*
 * Fragment grid of an h x w frame under p: *nbx fragment columns, *nby rows.
 * Host-only arithmetic, no device work.
 */
fov_status foveate_grid(int32_t h, int32_t w, const fov_params* p, int32_t* nbx, int32_t* nby);

/*
 * Geisler-Perry blur model (Appendix "Choosing the Standard Deviation", Eqs.
 * 2-6) as ramp parameters.  With CT0 = 1/64, alpha = 0.106 and e2 = 2.3 (the
 * constants the paper adopts), the cutoff f_c_deg(e) = e2 ln(1/CT0) /
 * (alpha (e + e2)) cycles/degree, f_c_pix = 0.5 f_c_deg / f_max cycles/pixel,
 * the eccentricity e = d / d_corner * e_corner degrees for a pixel distance d
 * from the fixation (d_corner = the half-diagonal of an h x w frame in
 * pixel-centre coordinates), and sigma = 1 / (2 pi f_c_pix).  That sigma is
 * affine in d, so it is written into p as the ramp's e0 (negative: every
 * fragment blurs, none is copied), slope and cap:
 *   sigma(d) = f_max alpha (e_corner d / d_corner + e2) / (pi e2 ln(1/CT0)),
 * capped at `cap` (> 0; use a large value for none).  f_max (cycles/degree at
 * the fovea) <= 0 selects f_c_deg(0), for which sigma(0) = 1/pi.  The other
 * fields of p (fixation, block, origin, sigma_map) are left as they are.
 * FOV_EINVAL for h, w < 1, a frame of one pixel, e_corner <= 0, a non-finite
 * argument or cap <= 0.  Host-only arithmetic.
 */
fov_status foveate_csf_params(int32_t h, int32_t w, double e_corner_deg, double f_max_cpd, double cap,
                              fov_params* p);

/*
 * Fragment shift (Alg. 1; Sec. 3 on the SSIM map): the tiling origin that
 * centres one fragment on the fixation, so that the copied fovea is as small
 * as possible and the blur moves with the gaze instead of snapping into place
 * at fragment boundaries.  Along each axis the fragment [s, s + B) with s the
 * integer nearest to fix - (B - 1)/2 (halves round up) has its midpoint within
 * half a pixel of the fixation; *origin_x / *origin_y receive s reduced into
 * (-B, 0].  block in 1..64 and a finite fixation, else FOV_EINVAL.  Host-only
 * arithmetic; copy the results into fov_params.origin_x / origin_y.
 */
fov_status foveate_fragment_shift(double fix_x, double fix_y, int32_t block, int32_t* origin_x,
                                  int32_t* origin_y);

/*
 * Per-fragment plan (the per-fragment blur strengths Alg. 1 sets up on the
 * host), computed ON THE
 * DEVICE by the same code the kernels run: sigma_out[by*nbx+bx] (double) and
 * r_out[...] (int32), both device arrays of nby*nbx entries owned by the
 * caller.  sigma_out may be NULL.  Asynchronous on `stream`.
 */
fov_status foveate_plan(int32_t h, int32_t w, const fov_params* p, double* sigma_out,
                        int32_t* r_out, void* stream);

/*
 * Same plan computed on the host (used for launch sizing and cost ordering);
 * host arrays of nby*nbx entries.  Not valid with a sigma_map (device data).
 */
fov_status foveate_plan_host(int32_t h, int32_t w, const fov_params* p, double* sigma_out,
                             int32_t* r_out);

/*
 * Foveate n frames: out = A_p(in) (Sec. 2; the device part of Alg. 1: the
 * padded fragment staged on chip, a horizontal pass, a vertical pass, the
 * store).
 *   in, out : same (n, c, h, w); dtype pairs u8->u8, u8->f32 (raw 0..255),
 *             f32->f32, f64->f64.  out must not overlap in (FOV_EALIAS).
 *   p       : np parameter sets, np == n (one per frame) or np == 1 (shared).
 *   stream  : hipStream_t (NULL = default stream).
 * Empty views (any extent 0) are a no-op.  Fails with FOV_ERANGE when a
 * fragment's radius needs more on-chip memory than one workgroup may use.
 * The library keeps a per-(device, stream) workspace for fragment plans (grown
 * with hipMalloc on first use or when a call needs more); calls on one stream
 * are ordered and may share it, calls on different streams use their own.
 */
fov_status foveate_forward(const fov_tensor* in, const fov_tensor* out, const fov_params* p,
                           int32_t np, void* stream);

/*
 * Foveate nframes frames of possibly different sizes in one launch: the
 * fragments of all frames form one queue, ordered by decreasing radius (their
 * cost), that a persistent grid drains (Alg. 1 run over a batch; each frame
 * keeps its own fixation and ramp).
 *   ins[i], outs[i] : views of one frame each (n == 1), any (c, h, w) and
 *                     strides; all frames share one dtype pair (as forward).
 *                     No output may overlap any input or another output.
 *   ps[i]           : parameters of frame i.
 * Frame descriptors beyond 16 are uploaded from a library-owned pinned buffer
 * to the library's per-stream workspace.  Asynchronous on `stream`; caller
 * buffers must stay alive until the stream reaches this work.
 */
fov_status foveate_forward_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps,
                                 int32_t nframes, void* stream);

/*
 * foveate_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and bitwise the same outputs as foveate_forward,
 * but the plan workspace is a fixed 16 MiB array of device memory that the
 * library's code object holds on every GPU it runs on until the process ends;
 * the call makes no hipMalloc, hipFree, pinned or other allocation.  Limits:
 *   - at most 16 frames per call (n <= 16; their descriptors travel in the
 *     kernel arguments), else FOV_EINVAL;
 *   - the call's plan workspace (per fragment about 4 * (2r_max + 1) bytes of
 *     taps plus a few words of queue) must fit the 16 MiB, else FOV_EINVAL
 *     with the size it needed; a 3840x2160 frame in 32 px fragments fits at
 *     every radius the on-chip memory allows.
 * Every call on one GPU uses that GPU's single array: calls that overlap on
 * the device (different streams, or host threads without ordering) race and
 * may produce wrong outputs; order them on one stream.  Nothing the array
 * keeps from an earlier call is read before it is rewritten.  The first call
 * on each device looks the array's device address up (hipGetSymbolAddress).
 */
fov_status foveate_forward_noalloc(const fov_tensor* in, const fov_tensor* out, const fov_params* p,
                                   int32_t np, void* stream);

/*
 * Adjoint (transpose) of foveate_forward for the same parameters:
 * grad_in = A_p^T grad_out, computed as a gather (each workgroup owns a tile
 * of grad_in and visits every fragment whose window reaches it; no atomics).
 * Used as the backward pass of training through the foveation.  dtype pairs
 * f32->f32 and f64->f64 only.  Same shape/alias/stream rules as forward.
 */
fov_status foveate_backward(const fov_tensor* grad_out, const fov_tensor* grad_in,
                            const fov_params* p, int32_t np, void* stream);

/* ---- launch tuning --------------------------------------------------------------------------
 *
 * How a forward launch maps fragments onto workgroups.  None of these choices
 * changes a result: every output pixel sums its taps in the same order, so
 * outputs are bitwise identical under every configuration.
 *   split      : each fragment is cut into split x split work items (output
 *                tiles of ceil(block / split) pixels a side, each staging its
 *                own halo); 1, 2 or 4.  Smaller tiles give more workgroups for
 *                small frames at the price of more halo work.
 *   strip_rows : rows of the padded tile (halo included) staged in LDS at
 *                once: 16, 32 or 64.  Fewer rows need less LDS per workgroup.
 *   persistent : 1 = a grid sized to what the chip holds at once strides
 *                over the work queue; 0 = one workgroup per queue slot.
 *   merge      : 1 = a fragment on an even row whose sigma and the sigma of
 *                the fragment below both equal the cap is one work item with
 *                it (equal taps: the halo rows the two share are computed
 *                once); needs split 1.  By default it is on unless its taller
 *                tiles would let fewer workgroups share a CU.
 *   chan_split : 1 = a fragment whose radius is at most 2/3 of the largest
 *                radius of the call is one work item per channel (such items
 *                come last in the queue and are latency bound: their channels
 *                then run side by side); needs split 1 and at most 16
 *                channels.  By default on for frames of several channels.
 *   time_us    : (output of foveate_autotune) median time of one call.
 */
typedef struct {
    int32_t split, strip_rows, persistent, merge, chan_split;
    float time_us;
} fov_tuning;

/*
 * Autotuner.  Runs foveate_forward (or foveate_forward_batch) with every
 * launch configuration that fits the device's LDS, `reps` timed calls each
 * (HIP events around the whole call on `stream`; 0 = 5), and stores the
 * fastest in the library's tuning cache under the call's workload class:
 * device architecture and CU count, dtype pair, channels, largest fragment
 * side, the bit length of the largest radius, the bit length of the fragment
 * count and the frame-count class (1, 2..16, more).  Later forward calls of
 * that class, from any thread, use the cached configuration; others use the
 * defaults (split 1, 64 strip rows, one workgroup per queue slot, merge and
 * chan_split as described above).  Writes
 * the chosen configuration to *best (may be NULL).  Arguments and errors as
 * foveate_forward / foveate_forward_batch; `out` holds the foveated frames on
 * return.  Synchronises `stream`.
 */
fov_status foveate_autotune(const fov_tensor* in, const fov_tensor* out, const fov_params* p, int32_t np,
                            int32_t reps, void* stream, fov_tuning* best);
fov_status foveate_autotune_batch(const fov_tensor* ins, const fov_tensor* outs, const fov_params* ps,
                                  int32_t nframes, int32_t reps, void* stream, fov_tuning* best);

/*
 * Force one configuration for the forward calls of the calling thread
 * (tests, experiments); NULL returns the thread to the cache and defaults.
 * FOV_EINVAL for values outside the sets above (or merge or chan_split 1 with
 * a split).  A forced configuration whose
 * LDS does not fit makes the forward call fail with FOV_ERANGE.
 */
fov_status foveate_tuning_force(const fov_tuning* t);

/* Empty the tuning cache. */
fov_status foveate_tuning_clear(void);

/* Number of entries in the tuning cache. */
fov_status foveate_tuning_count(int32_t* n);

/*
 * Write the tuning cache to a text file (one entry per line), or merge such a
 * file into it.  FOV_EINVAL (with the line number) for a malformed line; the
 * cache is left unchanged then.
 */
fov_status foveate_tuning_save(const char* path);
fov_status foveate_tuning_load(const char* path);

/* ---- serving -------------------------------------------------------------------------------
 *
 * A request loop for frames that arrive one at a time (each with its own
 * size and gaze), in the spirit of the paper's per-frame asynchronous loop
 * (the per-frame loop of Alg. 1), with continuous batching: a scheduler thread
 * admits queued frames while the bytes of admitted, unfinished frames stay
 * within an HBM budget, launches everything admitted as one batched forward
 * (the queue of foveate_forward_batch) on one of several streams, and admits
 * and launches frames that arrive while other batches are on the device, so
 * consecutive batches overlap on the GPU.  Frames stay where the caller put
 * them (device memory); results are identical to foveate_forward's.
 */
typedef struct fov_server fov_server;

typedef struct {
    size_t hbm_budget_bytes;      /* inputs + outputs of admitted, unfinished frames (> 0)      */
    int32_t max_batch_frames;     /* frames per batch, 1..4096                                  */
    int32_t max_inflight_batches; /* batches on the device at once, 1..8 (one stream each)      */
    int32_t max_requests;         /* request table size: queued + in flight + done, not polled  */
    int32_t in_dtype, out_dtype;  /* the one dtype pair this server serves (as forward)         */
    int32_t max_fragments;        /* fragments per batch (sizes the plan workspace)             */
    int32_t max_block;            /* largest fragment side a request may use (1..64)            */
    double max_sigma;             /* largest sigma a request may produce (sizes LDS and taps)   */
    int32_t use_graph;            /* 1: every batch replays a hipGraph captured at creation     */
    int32_t test_fake_device_us;  /* test hook: > 0 launches no kernels and completes each
                                     batch after this many microseconds (outputs untouched)     */
    int32_t test_fail_every;      /* test hook: every k-th batch completes with FOV_EHIP        */
    int32_t shared_stream;        /* 1: every in-flight batch queues on one stream (FIFO on the
                                     device, as a plain per-frame loop); 0: one stream per batch,
                                     in-flight batches run side by side                         */
} fov_server_cfg;

typedef struct {
    double t_submit, t_admit, t_launch, t_done; /* foveate_now() clock, seconds            */
    int32_t batch_frames;                        /* frames in the batch this one ran in     */
    int32_t status;                              /* fov_status of the frame's batch         */
} fov_timing;

/* Monotonic host clock (seconds) used for every server timestamp. */
double foveate_now(void);

/*
 * Create a server on the current device: streams, the scheduler thread and,
 * with use_graph, one captured batch graph per stream with its own workspace
 * (allocated here, sized by max_batch_frames, max_fragments, max_block and
 * max_sigma).  FOV_EINVAL for bad configuration, FOV_ENOMEM, FOV_EHIP.
 */
fov_status foveate_server_create(const fov_server_cfg* cfg, fov_server** out);

/*
 * Queue one frame: in, out are single-frame views (n == 1) of the server's
 * dtype pair; p its parameters (block <= max_block, every fragment's sigma
 * <= max_sigma, at most max_fragments fragments).  The buffers (and a sigma
 * map, if any) must stay alive until poll reports the ticket done.
 *   ready : a hipEvent_t that the caller recorded on the stream that produces
 *           `in` (and last used `out`), after that work; the frame's batch
 *           waits for it on the device before reading `in`.  The server's
 *           streams are not ordered after any caller stream, so without it
 *           `in` must already be complete on the device when the frame is
 *           submitted.  NULL = no wait.  The event must not be recorded again
 *           before poll reports the ticket done.
 * Returns with *ticket without waiting for the GPU; when a stream is free and
 * no frame is queued, the frame's batch is launched from the calling thread
 * before returning (the server's device is made current for that and
 * restored).  FOV_EAGAIN: request table full (poll and retry);
 * FOV_ECLOSED: the server is being destroyed; FOV_EINVAL / FOV_ERANGE /
 * FOV_EDTYPE / FOV_EALIAS as for forward, or a frame larger than the budget.
 */
fov_status foveate_submit(fov_server* s, const fov_tensor* in, const fov_tensor* out, const fov_params* p,
                          void* ready, uint64_t* ticket);

/*
 * *done = 1 once the frame's output is complete (then the ticket is retired
 * and *t, if not NULL, holds its timestamps), else 0.  Returns the frame's
 * status when done (FOV_OK, or the error its batch hit), FOV_OK while
 * pending, FOV_ENOTICKET for an unknown or retired ticket.
 */
fov_status foveate_poll(fov_server* s, uint64_t ticket, int32_t* done, fov_timing* t);

/*
 * Completion timestamp on the server clock: enqueue on `stream` a host
 * function that stores foveate_now() into *out when the stream reaches it
 * (used to time plain per-frame launches like served frames).  *out is host
 * memory owned by the caller and must stay valid until then.
 */
fov_status foveate_stream_timestamp(void* stream, double* out);

/* Block until every queued frame is done; tickets stay pollable. */
fov_status foveate_server_drain(fov_server* s);

/* Finish all queued work, stop the scheduler, release everything. */
fov_status foveate_server_destroy(fov_server* s);

/* ---- host-to-host pipeline ------------------------------------------------------------------
 *
 * Frames that live in host memory: each is uploaded, foveated and downloaded
 * (the per-frame loop of Alg. 1 moves the frame from pinned host memory to the
 * GPU and the result back; Sec. 3 gives the transfer time beside the kernel
 * time).  The upload of one frame, the foveation of the frame before it and
 * the download of the one before that overlap: the pipeline owns `depth`
 * device slots (one input and one output buffer each) and three streams
 * (upload, foveation, download), and frame k uses slot k mod depth, ordered
 * by events so that a slot is reused only after its previous frame has been
 * read out of it.  Results are identical to foveate_forward's.
 */
typedef struct fov_pipeline fov_pipeline;

/*
 * Create a pipeline on the current device with `depth` slots (1..16) whose
 * device buffers hold frames of up to max_in_bytes (input) and max_out_bytes
 * (output).  The buffers and streams are allocated here.  FOV_EINVAL,
 * FOV_ENOMEM, FOV_EHIP.
 */
fov_status foveate_pipeline_create(int32_t depth, size_t max_in_bytes, size_t max_out_bytes,
                                   fov_pipeline** out);

/*
 * Queue one frame.  host_in, host_out: single-frame views (n == 1) of HOST
 * memory, each dense (its elements fill one block from its first element, in
 * any order of the dims: HWC and CHW frames alike), dtype pairs as forward,
 * no overlap.  Pinned memory (hipHostMalloc, torch's pin_memory) lets the
 * copies overlap with other work; pageable memory is accepted, its copies
 * then hold the calling thread.  host_in must stay unchanged and host_out
 * alive until the ticket is done.  Returns with *ticket once the frame's
 * copies and kernels are queued.  FOV_EINVAL (also for a frame larger than
 * the buffers), FOV_ELAYOUT (a view that is not dense), FOV_EDTYPE,
 * FOV_EALIAS, FOV_ERANGE as for forward.
 */
fov_status foveate_pipeline_submit(fov_pipeline* pl, const fov_tensor* host_in, const fov_tensor* host_out,
                                   const fov_params* p, uint64_t* ticket);

/* *done = 1 once host_out holds the ticket's frame, else 0 (no wait).  FOV_ENOTICKET. */
fov_status foveate_pipeline_query(fov_pipeline* pl, uint64_t ticket, int32_t* done);

/* Block until host_out holds the ticket's frame, then retire the ticket.  FOV_ENOTICKET. */
fov_status foveate_pipeline_wait(fov_pipeline* pl, uint64_t ticket);

/* Finish all queued frames and release the pipeline's buffers and streams. */
fov_status foveate_pipeline_destroy(fov_pipeline* pl);

/*
 * Kernel timing for measurement.  Between foveate_profile_begin(capacity) and
 * foveate_profile_end(), each forward call made by this thread records the
 * start and end of its main kernel (the per-fragment blur; the plan and order
 * kernels that precede it are not included) in a pair of HIP events that the
 * kernel's dispatch stamps on its stream, up to `capacity` calls.  foveate_profile_end waits for the
 * recorded events, writes up to `capacity` durations in milliseconds to ms
 * (host array, may be NULL), stores how many in *count and releases the
 * events.  FOV_EINVAL if profiling was not started.
 */
fov_status foveate_profile_begin(int32_t capacity);
fov_status foveate_profile_end(float* ms, int32_t capacity, int32_t* count);

/*
 * Record only one forward call in `every` (the 1st, every+1-th, ...) of the
 * profile window started by foveate_profile_begin on this thread (default 1):
 * the calls in between run without events.  The main kernel's events are
 * stamped by its dispatch, which then does not overlap the next kernel of the
 * stream; sampling keeps that cost off most calls of a throughput run.
 * FOV_EINVAL if every < 1 or profiling was not started.
 */
fov_status foveate_profile_every(int32_t every);

/* Thread-local message for the last non-OK status of this thread ("" if none). */
const char* foveate_last_error(void);

/* Library version string. */
const char* foveate_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FOVEATE_H */
