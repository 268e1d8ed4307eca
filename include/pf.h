/*
 * pf.h -- C ABI of libpf, a particle filter for tracking an object in a
 * greyscale video, with its per-frame step written in HIP for AMD gfx950.
 *
 * The method is the bootstrap sampling-importance-resampling (SIR) particle
 * filter of Schieffer et al., "Boosting the Performance of Object Tracking with
 * a Half-Precision Particle Filter on GPU" (arXiv:2308.00763):
 *   Sec. 2   -- the three stages per time step (propagate, weight, resample);
 *   Sec. 4   -- Eq. (1)-(2) transition model, Eq. (3)-(4) log-likelihood over
 *               the pixels around a particle, the maximum, Eq. (5) weights,
 *               normalisation into a cumulative distribution, systematic
 *               resampling, and the precision variants (double, single, half);
 *   Sec. 5   -- the workload: a disk moving over a flat background with
 *               Gaussian noise.
 *
 * Conventions shared by every call:
 *   - Coordinates are in pixels; x is the column, y is the row.  A particle at
 *     (x, y) looks at pixel (floor(x + 1/2), floor(y + 1/2)).
 *   - Frames are H x W uint8 in device memory, row-major, `row_pitch` bytes
 *     between rows (row_pitch >= W).
 *   - The library never allocates device memory.  The caller allocates the
 *     workspace (pf_workspace_bytes) and owns it; a filter handle must not
 *     outlive its workspace.
 *   - All device work of a filter is ordered on the HIP stream given at
 *     pf_init; calls return before that work finishes unless stated.
 *   - Every function returns PF_OK (0) or a pf_status code; the text of the
 *     last error on the calling thread is available from pf_last_error().
 *     No C++ exception crosses this interface.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_ABI_VERSION 6

typedef enum pf_status {
    PF_OK = 0,
    PF_ERR_INVALID_ARG = 1, /* a parameter or pointer is out of its documented range */
    PF_ERR_WORKSPACE = 2,   /* the workspace is smaller than pf_workspace_bytes() */
    PF_ERR_HIP = 3,         /* a HIP runtime call failed; the handle is poisoned */
    PF_ERR_STATE = 4        /* the handle is poisoned by an earlier PF_ERR_HIP */
} pf_status;

/* Arithmetic precision of the step (paper Sec. 4, implementation paragraph:
 * one filter templated over double, float and half).
 *   PF_F64  -- positions, log-likelihoods, weights and the cumulative
 *              distribution in double; the baseline.
 *   PF_F32  -- positions in float (offsets from an integer origin), weights,
 *              normaliser and distribution in float; the distribution's
 *              carried tile offsets in compensated (two-float) arithmetic.
 *   PF_F16  -- positions in half (offsets from an integer origin), propagated
 *              with packed half arithmetic, two particles per 32-bit register;
 *              normaliser, distribution and estimate as in PF_F32.
 *   PF_BF16 -- positions in bfloat16 (offsets from an integer origin),
 *              propagated in float and rounded once to bfloat16; the rest as
 *              in PF_F32. */
typedef enum pf_dtype { PF_F64 = 0, PF_F32 = 1, PF_F16 = 2, PF_BF16 = 3 } pf_dtype;

/* Normalisation of the log-likelihood, Eq. (3): the sum over the N_d disk
 * pixels is divided by kappa * N_d (PF_LIK_MEAN, the paper's reading) or by
 * kappa alone (PF_LIK_SUM). */
typedef enum pf_lik_norm { PF_LIK_MEAN = 0, PF_LIK_SUM = 1 } pf_lik_norm;

/* Keep the per-particle diagnostics of the last step (weights before
 * resampling, ancestors, disk sums) so that pf_export / pf_export_step can
 * return them.  Costs extra workspace and memory traffic; off by default. */
#define PF_FLAG_DIAGNOSTICS 1u

/* Implementation variants, for measuring what the optimised step gains over
 * the straightforward one (paper Sec. 5: naive and optimised half-precision
 * kernels, and the threads-per-block study).  Every variant computes the
 * same step; results agree with the default up to the rounding of the
 * distribution.  Not accepted by the batch calls.
 *   PF_FLAG_NAIVE_LIKELIHOOD -- disk sums read every disk pixel from the frame
 *       (no LDS row-prefix table).
 *   PF_FLAG_NAIVE_RESAMPLE   -- the normalised cumulative distribution is
 *       written out (one division per particle; double in PF_F64, float
 *       otherwise), then one thread per slot binary-searches it, instead of
 *       the tile-wise slot fill.  Costs N more elements of workspace.
 *   Threads per workgroup, as a field value v in 1..5 selecting 2^(v+5)
 *   threads (64, 128, 256, 512, 1024; 0 = the default):
 *     bits 8-11 (PF_THREADS_A_SHIFT)  pass A, 1024 particles per workgroup:
 *                                     128, 256 (default) or 512 threads;
 *     bits 12-15 (PF_THREADS_C_SHIFT) pass C or the naive resampler: 64-1024
 *                                     (default 256 for both). */
#define PF_FLAG_NAIVE_LIKELIHOOD 2u
#define PF_FLAG_NAIVE_RESAMPLE 4u
/*   PF_FLAG_NAIVE_HALF       -- PF_F16 only, with the default pass-A size:
 *       the propagation runs one particle at a time in scalar half
 *       arithmetic (each normal cast to half on its own, a scalar half
 *       multiply-add and add per axis) instead of two particles per packed
 *       register; the same roundings, so the same results bit for bit.
 *       With PF_FLAG_NAIVE_RESAMPLE it is the straightforward half step the
 *       paper starts from (Sec. 4, pipeline-optimisation paragraph): no
 *       packing, and a division per particle and casts in the resampler. */
#define PF_FLAG_NAIVE_HALF (1u << 29)
#define PF_THREADS_A_SHIFT 8
#define PF_THREADS_C_SHIFT 12

/* Metropolis resampling (Murray, Lee & Jacob, 2016; among the scan-free
 * resamplers of the paper's related work, Sec. 3) instead of systematic
 * resampling: slot j runs a chain of B steps that starts at particle j; each
 * step proposes a particle i uniformly and moves there when
 * u <= w_i / w_k = exp(L_i - L_k) (always when L_i >= L_k).  No maximum,
 * normaliser or cumulative distribution enters the resampling (the estimate
 * still uses them); the result is biased for finite B, the bias falling
 * geometrically with B.  Random numbers: steps 2m and 2m + 1 of slot j at
 * step t use counter (j, t, stream_id, 2 + m), words 0-1 and 2-3; the first
 * of each pair picks i = floor(word * N / 2^32), the second gives u =
 * (word + 1/2) 2^-32 (the top 24 bits in the reduced modes).  B in bits 18-25
 * (PF_METROPOLIS_STEPS_SHIFT; 0 = 32).  Costs 4 bytes per particle of
 * workspace.  Not accepted by the batch calls. */
#define PF_FLAG_METROPOLIS (1u << 16)
#define PF_METROPOLIS_STEPS_SHIFT 18

/* Multinomial resampling by the Gumbel-max scheme (the alternative weighed
 * in the paper, Sec. 4, numerical-stability paragraph) instead of systematic
 * resampling: slot i takes argmax_j (L_j + G_ij) with G_ij = -ln(-ln u)
 * standard Gumbel noise, u = (word + 1/2) 2^-32 (the top 24 bits in the
 * reduced modes), the word j mod 4 of Philox at counter (floor(j/4), i, t,
 * stream_id) under key (seed low, seed high xor 0x47756D62).  It works on
 * the unnormalised log weights but draws N^2 noise values per step, so it
 * accepts N <= 65536 (the paper's particle limit).  Costs 4 bytes per
 * particle of workspace.  Not accepted by the batch calls. */
#define PF_FLAG_GUMBEL_MAX (1u << 17)

/* Rejection resampling (Murray, Lee & Jacob, 2016; the other scan-free
 * resampler of the paper's related work, Sec. 3) instead of systematic
 * resampling: slot j first proposes particle j; a proposal c is accepted
 * with probability w_c / w_max = exp(L_c - max L), and after a rejection the
 * next proposal is a uniform particle.  Each particle's expected offspring
 * count is exactly N w_c (unbiased) while no slot runs out of trials; at
 * most 64 v trials (v in bits 18-25, PF_METROPOLIS_STEPS_SHIFT; 0 = 4096),
 * after which a slot keeps its last proposal.  Needs the maximum but no
 * normaliser or cumulative distribution.  Random numbers: trials 2q and
 * 2q + 1 of slot j at step t use counter (j, t, stream_id, 2 + q), words 0-1
 * and 2-3; the first of each pair gives u = (word + 1/2) 2^-32 (the top 24
 * bits in the reduced modes), the second the next proposal
 * floor(word * N / 2^32).  Costs 4 bytes per particle of workspace.  Not
 * accepted by the batch calls. */
#define PF_FLAG_REJECTION (1u << 28)

/* A filter whose workspace holds only its state: the device block (step
 * count, origins, estimate), the particle positions and, with
 * PF_FLAG_DIAGNOSTICS, the diagnostics -- 2 * elt bytes per particle plus
 * 256 instead of about 5 * elt.  Its steps run through
 * pf_step_static_scratch, whose per-step scratch (tile records and table,
 * propagated positions, tile prefix sums) is the library's static device
 * array, shared by every such filter on the device.  Accepted only with the
 * default step (no PF_FLAG_NAIVE_*, PF_FLAG_METROPOLIS, PF_FLAG_GUMBEL_MAX or
 * PF_FLAG_REJECTION) and only when that scratch fits PF_STATIC_SCRATCH_BYTES
 * (N <= 2^20 in PF_F64, about 2.09 million in PF_F32, 3.1 million in PF_F16
 * and PF_BF16); not accepted by the batch calls.  pf_step and the
 * propagated positions of pf_export_step refuse such a filter. */
#define PF_FLAG_STATE_ONLY (1u << 26)

/* Workgroup sizes from the tuning table (the threads-per-block study of the
 * paper's Sec. 5, kept per GPU): pf_init, pf_batch_init and pf_batch_reinit
 * replace both threads fields with the entry that the table installed in the
 * library (pf_tune_set, pf_tune_load) holds for the stream's GPU
 * architecture, the dtype and the particle-count bucket ceil(log2 N), as
 * pf_tune_lookup resolves it; the defaults when the table has nothing for
 * that architecture and dtype.  Both threads fields must be 0, and
 * PF_FLAG_NAIVE_HALF (which runs pass A at its default size) is refused with
 * it.  pf_launch_config reports the sizes a filter resolved to.  The sizes
 * change results only through pass A's, which fixes the order of the
 * tile-local prefix sums. */
#define PF_FLAG_TUNED (1u << 30)

/* Size of the static step scratch (bytes per device). */
#define PF_STATIC_SCRATCH_BYTES (24u * 1024u * 1024u + 64u * 1024u)

typedef struct pf_params {
    uint32_t struct_size;  /* must be sizeof(pf_params) */
    int32_t dtype;         /* pf_dtype */
    int64_t n_particles;   /* N, 1 <= N <= 2^28 */
    int32_t width;         /* W, frame columns, > 2 * disk_radius */
    int32_t height;        /* H, frame rows, > 2 * disk_radius */
    int32_t disk_radius;   /* r, 1 <= r <= 32; pixels with dx^2 + dy^2 < r^2 */
    int32_t fg;            /* foreground intensity (paper: 228), 0..255 */
    int32_t bg;            /* background intensity (paper: 100), 0..255 */
    int32_t lik_norm;      /* pf_lik_norm */
    double kappa;          /* likelihood scale (paper: 50), > 0 */
    double x0, y0;         /* initial object position; every particle starts here */
    double drift_x;        /* mean displacement per frame, Eq. (1): 1.0 */
    double drift_y;        /* Eq. (2); -2.0 for an object moving toward y = 0 */
    double sigma_x;        /* transition standard deviation, Eq. (1): 5.0 */
    double sigma_y;        /* Eq. (2): 2.0 */
    uint64_t seed;         /* key of the counter-based random streams */
    uint32_t stream_id;    /* filter id inside the random-stream counter */
    uint32_t flags;        /* PF_FLAG_* */
} pf_params;

typedef struct pf_filter pf_filter;

/* Device bytes a filter with these parameters needs (pf_init).  Pure
 * function: touches no device.  Errors: PF_ERR_INVALID_ARG for out-of-range
 * parameters or a NULL pointer. */
int pf_workspace_bytes(const pf_params* p, size_t* out_bytes);

/* Device bytes a batch member with these parameters needs (a share for
 * pf_batch_rebind): pf_workspace_bytes less what only a filter of its own
 * uses (the buffers of the deferred resampling, see pf_step).  Pure
 * function.  Errors as pf_workspace_bytes. */
int pf_member_bytes(const pf_params* p, size_t* out_bytes);

/* Initialisation (paper Sec. 4, Fig. 1: the filter starts after an
 * initialization phase): all N particles at (x0, y0) with weight 1/N, step
 * counter t = 0.  `d_workspace` is device memory of at least
 * pf_workspace_bytes() bytes, 256-byte aligned, owned by the caller;
 * `hip_stream` is a hipStream_t (NULL for the default stream).  On success
 * *out receives a host handle (freed by pf_destroy).
 * Errors: PF_ERR_INVALID_ARG, PF_ERR_WORKSPACE, PF_ERR_HIP. */
int pf_init(const pf_params* p, void* d_workspace, size_t workspace_bytes, void* hip_stream,
            pf_filter** out);

/* One SIR step on one frame (paper Sec. 2 three stages; Sec. 4 six kernels):
 * t <- t + 1; every particle k draws two normals from random stream
 * (k, t, stream_id) and moves by (drift + sigma * z) (Eq. (1)-(2)); its
 * log-likelihood is the disk sum of Eq. (3) over `d_frame`; weights are
 * exp(L - max L) (Eq. (5), previous weights are all 1/N after resampling);
 * the weighted mean position before resampling becomes the estimate; the
 * normalised cumulative weights are resampled systematically with the offset
 * drawn from stream (0, t, stream_id, purpose 1) (Sec. 4, resampling
 * paragraph).  An FP64 or FP32 filter of at most 2^20 particles resampling
 * systematically, without diagnostics or measurement variants, at the default
 * pass-A and pass-C sizes, defers the resampling of each step into the next
 * step, whose first kernel
 * gathers the resampled particles for its tiles (two kernels per step instead
 * of three); pf_export runs a pending resampling first, and every result is
 * bit-identical to resampling at once.  Asynchronous on the filter's stream; `d_frame` must stay valid
 * until the step has run.  The call enqueues kernels only (no host wait,
 * allocation or memset), so it may be captured into a HIP graph by stream
 * capture on the filter's stream: the step count lives on the device, and
 * each replay advances the filter by one step on the frame at the pointer
 * given at capture (refill that buffer between replays).  Errors:
 * PF_ERR_INVALID_ARG (NULL frame, pitch < W), PF_ERR_HIP (the handle is then
 * poisoned), PF_ERR_STATE. */
int pf_step(pf_filter* h, const uint8_t* d_frame, int64_t row_pitch);

/* The step of pf_step for a filter created with PF_FLAG_STATE_ONLY, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): it allocates nothing and needs no
 * scratch from the caller.  The scratch of the step is a static device array
 * of PF_STATIC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends (its address is looked up once per device, in
 * pf_init of the first such filter on that device).  The step's kernels and
 * arithmetic are those of pf_step: its results are bit-identical to pf_step
 * on a filter with the same parameters, frames and step count.
 * Every call on a device shares that device's array: calls that may overlap
 * on one device (different streams without ordering between them) race and
 * give wrong results; order them on one stream or synchronise.  Nothing of
 * the array needs clearing between calls (each step writes every scratch
 * word it reads).  Errors: PF_ERR_INVALID_ARG (not a PF_FLAG_STATE_ONLY
 * filter, NULL frame, pitch < W, a stream on another device than the one the
 * filter was created on), PF_ERR_HIP (the handle is then poisoned),
 * PF_ERR_STATE. */
int pf_step_static_scratch(pf_filter* h, const uint8_t* d_frame, int64_t row_pitch);

/* The estimate of the latest step (x, y in pixels), or (x0, y0) before the
 * first step.  Waits for the filter's stream.  Errors: PF_ERR_STATE,
 * PF_ERR_HIP, PF_ERR_INVALID_ARG (NULL out). */
int pf_estimate(pf_filter* h, double out_xy[2]);

/* Stream-ordered copy of the latest estimate into device memory
 * (`d_out_xy`: 2 doubles, device pointer); does not wait. */
int pf_estimate_async(pf_filter* h, double* d_out_xy);

/* Copy the filter's state to host memory (waits for the stream; a pending
 * resampling of the latest step, see pf_step, is run first when x or y is
 * requested).  Each pointer may be NULL to skip it; arrays hold N elements.
 *   x, y    -- particle positions after the latest resampling (the next
 *              step's ancestors), in absolute pixels;
 *   w_norm  -- normalised weights of the latest step before resampling, in
 *              particle order of that step (needs PF_FLAG_DIAGNOSTICS);
 *   anc     -- ancestor of every slot of the latest resampling
 *              (needs PF_FLAG_DIAGNOSTICS);
 *   t       -- steps taken (the device's count, so replays of a captured
 *              pf_step are included).
 * Errors: PF_ERR_INVALID_ARG (diagnostics requested without the flag, or no
 * step taken yet for w_norm/anc), PF_ERR_STATE, PF_ERR_HIP. */
int pf_export(pf_filter* h, double* x, double* y, double* w_norm, int32_t* anc, uint32_t* t);

/* The propagated positions and disk sums of the latest step, before
 * resampling, in absolute pixels (needs PF_FLAG_DIAGNOSTICS for disk_sum; the
 * positions are always available after a step).  disk_sum[k] is the integer
 * sum over the disk of (I - bg)^2 - (I - fg)^2.  Any pointer may be NULL. */
int pf_export_step(pf_filter* h, double* x_prop, double* y_prop, int32_t* disk_sum);

/* Replace the particle positions (host arrays of N doubles, absolute pixels)
 * and the step counter; weights become 1/N (a pending resampling of the
 * latest step, see pf_step, is discarded).  Used for checkpoint/resume and
 * teacher-forced comparisons.  Reduced-precision modes round each position
 * to the mode's storage precision.  Stream-ordered; waits for the copy. */
int pf_import(pf_filter* h, const double* x, const double* y, uint32_t t);

/* Free the host handle (not the workspace).  NULL is accepted. */
int pf_destroy(pf_filter* h);

/* Text of the last error on the calling thread; valid until the next libpf
 * call on that thread.  Never NULL. */
const char* pf_last_error(void);

/* Per-pass timing with HIP events on the filter's stream.  pf_profile_start
 * creates the events for up to `max_steps` steps (host-side objects, no device
 * memory); the following pf_step calls launch their kernels with start and
 * stop events stamped by each kernel's own dispatch (its execution time, no
 * extra queue packets); pf_profile_read waits for the stream and returns the
 * summed durations in milliseconds: out_ms[0] = pass A (propagate, likelihood, tile
 * maximum, weights, tile prefix sums), out_ms[1] = combine (global maximum,
 * normaliser, carried offsets, estimate, resampling offset), out_ms[2] = pass C
 * (systematic-resampling scatter; 0 for a filter that defers its resampling,
 * see pf_step: pass A gathers it), and the number of steps recorded; it then
 * stops recording and frees the events.  Errors: PF_ERR_INVALID_ARG,
 * PF_ERR_HIP. */
int pf_profile_start(pf_filter* h, uint32_t max_steps);
int pf_profile_read(pf_filter* h, double out_ms[3], uint32_t* steps);

/* ------------------------------------------------------------------------
 * Tuning table: (GPU architecture, dtype, particle-count bucket) -> (pass-A
 * threads, pass-C threads), read by PF_FLAG_TUNED.  One table per process,
 * shared by every device and thread (the calls take a lock); entries persist
 * as a text file that pf_tune_load reads (the package ships one measured on
 * its target GPU).
 */

/* Install entry (arch, dtype, bucket), replacing one with the same key.
 * arch: architecture name without feature suffixes ("gfx950"), 1 to 31
 * characters of [A-Za-z0-9_]; bucket b in [0, 28] covers the particle
 * counts N with ceil(log2 N) = b; threads_a in {0, 128, 256, 512} and
 * threads_c in {0, 64, 128, 256, 512, 1024}, 0 meaning the default size.
 * Errors: PF_ERR_INVALID_ARG (nothing changes). */
int pf_tune_set(const char* arch, int32_t dtype, int32_t bucket, int32_t threads_a, int32_t threads_c);

/* Read a table file (text, one entry a line: `arch dtype bucket threads_a
 * threads_c`, dtype one of f64 f32 f16 bf16; blank lines and anything after
 * '#' ignored) and install its entries as pf_tune_set does.  The whole file
 * is checked first: a bad line installs nothing.  *out_entries (may be NULL)
 * receives the number of entries read.  Errors: PF_ERR_INVALID_ARG (file
 * unreadable, or the text names the first bad line). */
int pf_tune_load(const char* path, int32_t* out_entries);

/* Remove every entry. */
int pf_tune_clear(void);

/* The sizes PF_FLAG_TUNED resolves to for architecture `arch`, `dtype` and n
 * particles: the entry of bucket ceil(log2 n), else the entry of the nearest
 * bucket with the same arch and dtype (the smaller bucket on a tie), else 0
 * and 0 (the defaults).  Host only.  Errors: PF_ERR_INVALID_ARG. */
int pf_tune_lookup(const char* arch, int32_t dtype, int64_t n, int32_t* threads_a, int32_t* threads_c);

/* The workgroup sizes filter h launches with: pass A threads (128, 256 or
 * 512) and pass C threads (the naive resampler's with
 * PF_FLAG_NAIVE_RESAMPLE; for a batch member, the batch's pass C size,
 * which it uses for every member).  Errors: PF_ERR_INVALID_ARG. */
int pf_launch_config(pf_filter* h, int32_t* threads_a, int32_t* threads_c);

/* ------------------------------------------------------------------------
 * Batches: many independent filters (one per video stream, say), each running
 * the step of pf_step (paper Sec. 2 and Sec. 4) on its own frame, advanced
 * together with one launch per pass.  The filters of a batch share the dtype;
 * everything else in their parameters may differ (N, frame size, radius,
 * seeds, motion model, pass-A size).  A filter's results in a batch are
 * bit-identical to the same filter run alone through pf_step with the same
 * parameters, frames and step count: each of its workgroups runs the
 * single-filter code on that filter's data, whatever else the batch holds.
 * Members may take PF_FLAG_DIAGNOSTICS, PF_FLAG_TUNED and the threads fields
 * (no other variant): pass A runs each member at its own size, one launch
 * per size present; pass C runs every member at the batch's size (the pass-C
 * size changes no result).
 */
typedef struct pf_batch pf_batch;

/* Device bytes for a batch of n filters (1 <= n <= 2^20) with parameters
 * ps[0..n-1], all of one dtype, at most 2^31 - 1 tiles of 1024 particles in
 * total.  Pure function.  Errors: PF_ERR_INVALID_ARG (the text names the
 * first offending filter). */
int pf_batch_workspace_bytes(const pf_params* ps, int32_t n, size_t* out_bytes);

/* Initialise every filter of the batch as pf_init does, inside one caller-
 * owned workspace (device memory, 256-byte aligned, at least
 * pf_batch_workspace_bytes() bytes; the batch must not outlive it).  The
 * batch allocates pinned host memory for staging each step's plan (32 bytes
 * per filter plus 8 bytes per tile, four copies: three for eager steps, one
 * for a captured step) and frees it in pf_batch_destroy.  All device work is ordered on `hip_stream`; waits for
 * the initialisation to finish.  Errors: PF_ERR_INVALID_ARG,
 * PF_ERR_WORKSPACE, PF_ERR_HIP. */
int pf_batch_init(const pf_params* ps, int32_t n, void* d_workspace, size_t workspace_bytes,
                  void* hip_stream, pf_batch** out);

/* One step of every filter k whose active[k] is non-zero (`active` NULL: all
 * filters) on frame d_frames[k] (device, H_k x W_k uint8, row pitch
 * pitches[k] >= W_k).  d_frames and pitches are host arrays of n entries;
 * entries of inactive filters are not read.  Continuous batching: the active
 * set may change from call to call.  Asynchronous on the batch's stream; the
 * frames must stay valid until the step has run.
 * HIP graphs: called while the batch's stream is being captured, the step is
 * recorded instead of run (no host wait, allocation or memset): the plan
 * (frame pointers, pitches, active set) goes to the staging copy kept for
 * captured steps, and every replay uploads it and advances each active
 * filter by one step on the frames at those pointers (refill them between
 * replays).  The batch keeps one captured plan: a later capture replaces the
 * plan that earlier captured graphs read, and so does a re-capture after
 * pf_batch_reinit (a graph captured before it steps the new filter with the
 * old plan: tiles past its new size are skipped, its results are
 * meaningless).  Eager steps and replays may be interleaved.  Errors: PF_ERR_INVALID_ARG (nothing is stepped), PF_ERR_HIP
 * (the batch and its filters are then poisoned), PF_ERR_STATE. */
int pf_batch_step(pf_batch* b, const uint8_t* const* d_frames, const int64_t* pitches,
                  const uint8_t* active);

/* The latest estimate of every filter: out_2n[2k], out_2n[2k + 1] = (x, y) of
 * filter k (host array of 2n doubles); (x0, y0) for a filter not yet stepped.
 * Waits for the stream. */
int pf_batch_estimates(pf_batch* b, double* out_2n);

/* The same into device memory (`d_out_2n`, 2n doubles), stream-ordered; does
 * not wait. */
int pf_batch_estimates_async(pf_batch* b, double* d_out_2n);

/* Re-initialise filter k of the batch in place with new parameters, as
 * pf_init does (particles at (x0, y0), t = 0): a continuous-batching server
 * hands the share of a finished stream to an arriving one.  The parameters
 * must have the batch's dtype and fit the filter's workspace share (the
 * bytes of the parameters it was created with, or of its last
 * pf_batch_rebind), and the members' tiles together must fit the batch's
 * plan (the members' tiles at creation, or pf_batch_init_cap's capacity).
 * Waits for the stream before and after.  Errors: PF_ERR_INVALID_ARG,
 * PF_ERR_WORKSPACE (the share or the plan is too small; nothing changes),
 * PF_ERR_HIP, PF_ERR_STATE. */
int pf_batch_reinit(pf_batch* b, int32_t k, const pf_params* p);

/* The two calls above with room in the batch's plan for max_tiles tiles in
 * total (at least the members' own tiles; 0 = exactly those), so that
 * members can later be rebound (pf_batch_rebind) to larger filters whose
 * workspace shares lie outside the batch workspace.  The plan costs 16 bytes
 * of workspace and 32 bytes of pinned host memory per tile of capacity.
 * Errors as for pf_batch_workspace_bytes and pf_batch_init (max_tiles outside
 * [0, 2^31 - 1]: PF_ERR_INVALID_ARG). */
int pf_batch_workspace_bytes_cap(const pf_params* ps, int32_t n, int64_t max_tiles, size_t* out_bytes);
int pf_batch_init_cap(const pf_params* ps, int32_t n, int64_t max_tiles, void* d_workspace,
                      size_t workspace_bytes, void* hip_stream, pf_batch** out);

/* Re-initialise filter k of the batch as pf_batch_reinit does, on a new
 * workspace share: share_bytes bytes of device memory at d_share (256-byte
 * aligned, at least pf_member_bytes(p); owned by the caller, who keeps it
 * valid and unshared while filter k is bound to it, i.e. until the next
 * rebind of k or pf_batch_destroy).  Lets a server hand its filters shares
 * from its own device-memory budget, sized per stream, instead of fixed
 * shares inside the batch workspace: after a rebind, pf_batch_reinit of k
 * reuses the new share.  The members' tiles together must stay within the
 * batch's plan capacity (pf_batch_init_cap).  Waits for the stream before and
 * after; a graph captured before steps the filter with the old plan (as after
 * pf_batch_reinit).  Errors: PF_ERR_INVALID_ARG, PF_ERR_WORKSPACE (the share
 * or the plan is too small; nothing changes), PF_ERR_HIP, PF_ERR_STATE. */
int pf_batch_rebind(pf_batch* b, int32_t k, const pf_params* p, void* d_share, size_t share_bytes);

/* Handle of filter k (0 <= k < n) of the batch, owned by the batch and valid
 * until pf_batch_destroy.  pf_estimate, pf_estimate_async, pf_export,
 * pf_export_step, pf_import, pf_step (which steps that filter alone) and the
 * profile calls accept it; pf_destroy refuses it (PF_ERR_INVALID_ARG). */
int pf_batch_filter(pf_batch* b, int32_t k, pf_filter** out);

/* Free the batch's host objects and its filters' handles (not the
 * workspace).  Waits for the stream.  NULL is accepted. */
int pf_batch_destroy(pf_batch* b);

/* PF_ABI_VERSION of the loaded library. */
int pf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
