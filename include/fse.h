/*
 * fse.h -- C ABI of the MI355X implementation of Frequency Selective
 * Extrapolation (FSE) with the optimized, parallel block processing order of
 * Seiler & Kaup, "Optimized and Parallelized Processing Order for Improved
 * Frequency Selective Signal Extrapolation".
 *
 * What the library computes (paper Section 2 and Section 3):
 *   An 8-bit image is divided into blocks (Section 2).  Every block holding
 *   lost samples is extrapolated from its extrapolation area L (the block plus
 *   a frame of d samples): the weighting function of Eq. (2) is applied, the
 *   model of Eq. (1) is generated from DFT basis functions (Section 4) by K
 *   greedy iterations (select the basis function with the largest weighted
 *   energy reduction, estimate its coefficient with orthogonality deficiency
 *   compensation factor gamma), and the model's samples are inserted into the
 *   lost part of the block.  Blocks are processed either in line-scan order
 *   (Section 2) or in waves of mutually non-adjacent blocks chosen by
 *   Algorithm 1 (Section 3, Eq. (3)) or by the refined sample-count
 *   criterion Section 3 suggests; the blocks of one wave run concurrently.
 *
 *   Readings of points the paper leaves open, fixed by this ABI:
 *   - basis phi_k[m,n] = exp(+j 2 pi (k1 m / fft_h + k2 n / fft_w)), L at the
 *     top-left of the fft_h x fft_w grid; the output is the real part;
 *   - selection = argmax over k of |P[k]|^2 (P = weighted DFT of the current
 *     residual), ties to the smallest k1*fft_w + k2; coefficient increment =
 *     gamma * P[u] / sum(w); exactly `iterations` iterations;
 *   - neighbours = 8-neighbourhood; rim blocks count their missing
 *     neighbours as not extrapolated (margin +3, corner +5); N_min is the
 *     smallest non-negative count; the wave is filled in raster order
 *     (the refined order counts unknown samples instead: FSE_ORDER_REFINED);
 *   - every block of a wave reads the image as it was at the start of the
 *     wave; reconstructed samples are reused unquantized;
 *   - lost output samples are rounded half-to-even and clamped to [0, 255].
 *
 * Threading: a plan is used by one host thread at a time, except that
 * fse_submit and fse_poll may be called concurrently with each other.
 * All functions return FSE_OK (0) or a negative FSE_ERR_* code; fse_poll may
 * also return FSE_PENDING.
 */
#ifndef FSE_H
#define FSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSE_OK 0
#define FSE_PENDING 1
#define FSE_ERR_INVALID (-1)     /* null pointer, parameter out of range */
#define FSE_ERR_UNSUPPORTED (-2) /* valid request this build cannot run */
#define FSE_ERR_NOMEM (-3)       /* can never fit the device memory budget */
#define FSE_ERR_AGAIN (-4)       /* serving slots full right now; retry */
#define FSE_ERR_DEVICE (-5)      /* HIP error; sticky for the plan */
#define FSE_ERR_TICKET (-6)      /* unknown or already consumed ticket */

typedef struct fse_plan_s *fse_plan_t; /* opaque, owned by the library */

/* Block processing order: Algorithm 1 (Section 3), line scan (Section 2), or
 * the refined criterion Section 3 suggests as an alternative: Algorithm 1
 * with N(b) counting the lost, not yet extrapolated samples of the 8
 * neighbouring blocks instead of the neighbouring blocks with losses (a
 * neighbour cell outside the image counts as a whole block of unknown
 * samples; a finished block's samples leave its neighbours' N).  With
 * whole-block losses the refined order equals Algorithm 1; with partial
 * losses it orders by sample counts, usually in more, smaller waves. */
enum { FSE_ORDER_OPTIMIZED = 0, FSE_ORDER_LINESCAN = 1, FSE_ORDER_REFINED = 2 };

/* Arithmetic of the per-block iteration.  Only FSE_FP64 and FSE_FP32_RERANK
 * reproduce the FP64 selection closely enough for a maximum sample error of
 * 0.5 on the 8-bit scale in every block; FSE_FP32 and FSE_FP32_F16X3 compute
 * their spectra in float, whose rounding (about 1e-7 of the largest spectrum
 * entry) decides a few near-tied selections differently (measured: a few
 * blocks in a hundred above 0.5, whole-image PSNR within 0.02 dB). */
enum {
  FSE_FP64 = 0,        /* spectra, weights, coefficients in double */
  FSE_FP32 = 1,        /* spectra and iteration in float; synthesis sums in double */
  FSE_FP32_RERANK = 2, /* transforms in double, iteration in float; whenever another
                          spectrum entry comes within rerank_gap (relative) of the
                          float maximum of |R|^2, every entry within that gap is
                          re-scored exactly in double (R0 - sum dc_i W[k - u_i], with
                          the increments dc_i as applied) and the largest exact value
                          is selected, ties to the smallest index; no candidate is
                          dropped (fse_call_stats counts them).  The float spectrum
                          is not re-scored once its maximum falls below 2^-40 of the
                          block's first maximum (rounding noise) */
  FSE_FP32_F16X3 = 3    /* iteration as FSE_FP32; both DFT stages as dense products
                          on matrix cores, every operand split into two f16 parts
                          (about 22 significant bits; three products each, float
                          accumulation); 4 wavefronts per block in every launch */
};

/* fse_params.flags */
#define FSE_FLAG_DEVICE_PTRS 1 /* frame pointers are device pointers */

typedef struct {
  int32_t block_w, block_h; /* block size in samples, 1..64 (paper: 2..16) */
  int32_t border_d;         /* frame width d around the block, >= 0 */
  int32_t fft_w, fft_h;     /* basis grid; this build supports 64 x 64 */
  double rho;               /* weighting decay of Eq. (2), in (0, 1] */
  double delta;             /* reconstructed-area weight of Eq. (2), [0, 1] */
  double gamma;             /* orthogonality deficiency compensation, (0, 1] */
  int32_t iterations;       /* K, 1..FSE_MAX_ITERATIONS */
  int32_t order;            /* FSE_ORDER_* */
  int32_t precision;        /* FSE_FP64, FSE_FP32, FSE_FP32_RERANK, FSE_FP32_F16X3 */
  int32_t grid_off_x;       /* block grid shift, 0 <= off < block size: */
  int32_t grid_off_y;       /*   block column j covers x in
                               [j*block_w - grid_off_x, +block_w) */
  double empty_fill;        /* value written when L has no support */
  int64_t device_mem_budget;   /* bytes for serving frames; 0 = 4 GiB */
  int32_t max_inflight_frames; /* serving slots; 0 = 64 */
  int32_t flags;               /* FSE_FLAG_* */
  double rerank_gap;           /* FSE_FP32_RERANK: relative gap, [0, 0.5); 0 = 1e-4 */
} fse_params;

#define FSE_MAX_ITERATIONS 1024

/* Per-frame statistics (filled when fse_frame.stats is not null). */
typedef struct {
  int32_t waves;            /* waves this frame needed */
  int32_t lost_blocks;      /* blocks holding at least one lost sample */
  int32_t max_wave_blocks;  /* largest wave of this frame */
  int32_t reserved;
  double latency_ms;        /* fse_submit -> completion (serving only) */
} fse_stats;

/* Per-block trace of the greedy iteration (filled when fse_frame.trace is
 * not null).  Arrays are caller-owned with room for `capacity` blocks.  */
typedef struct {
  int32_t capacity;     /* in: slots available */
  int32_t count;        /* out: lost blocks of the frame (may exceed capacity;
                           only the first `capacity` are written) */
  int32_t *block;       /* [capacity] block index bi * wb + bj */
  int32_t *wave;        /* [capacity] wave of that block */
  int32_t *u;           /* [capacity * iterations] selected k1*fft_w + k2 */
  double *dc;           /* [capacity * iterations * 2] (re, im) increments */
} fse_trace;

typedef struct {
  const uint8_t *image; /* height rows of `stride` bytes; lost values ignored */
  int32_t width, height, stride;
  const uint8_t *lost;  /* nonzero = lost sample */
  int32_t lost_stride;
  uint8_t *out;         /* result, may alias image; known samples copied */
  int32_t out_stride;
  float *out_f32;       /* nullable: unquantized result as float, width*height
                           contiguous (known samples hold their input value) */
  double *out_f64;      /* nullable: the same as double */
  fse_trace *trace;     /* nullable, host memory */
  fse_stats *stats;     /* nullable, host memory */
} fse_frame;

/*
 * Create a plan: validates the parameters, allocates the per-plan tables on
 * the current HIP device and takes the stream (a hipStream_t, nullable = the
 * library's own stream; with FSE_FLAG_DEVICE_PTRS this should be the caller's
 * stream so that device buffers are ordered with the caller's work).
 * Errors: FSE_ERR_INVALID (p or out null, parameter out of range,
 * block + 2d > fft), FSE_ERR_UNSUPPORTED (fft other than 64 x 64),
 * FSE_ERR_DEVICE (no usable device).  On error *out is set to NULL.
 * Tuning: environment variables read here.  FSE_WAVE_THRESHOLDS="t16,t8"
 * sets the launch sizes (blocks per launch) up to which a block runs on 16
 * or on 8 wavefronts instead of 4; results equal the oracle's to the same
 * tolerance in every shape, not bit for bit across shapes.
 * FSE_FRAME_GROUPS=g (1..16) sets the number of frame groups of a batched
 * call (default 3).  FSE_CRIT_DEPTH=c (0..1): frames whose schedule has at
 * least c times the waves of the deepest frame form a group of their own,
 * whose workgroups raise their wave priority (FSE_CRIT_PRIO=0 keeps the
 * default priority); 0 = off, default 0.9.  FSE_CRIT_WAVES=w (4, 8 or 16;
 * 0 = by that group's launch size) sets the wavefronts per block of that
 * group (default 4).  None of these changes results
 * beyond the per-shape rounding noted above.
 */
int32_t fse_plan(const fse_params *p, void *hip_stream, fse_plan_t *out);

/* Destroy a plan: cancels queued serving frames, waits for in-flight work and
 * frees every device and host resource.  NULL is accepted. */
int32_t fse_plan_destroy(fse_plan_t plan);

/*
 * Conceal n frames synchronously (paper Section 2-3 as described above).
 * n > 1 batches the frames: wave t of the call is the union of wave t of every
 * frame, executed as one kernel launch, so each frame gets exactly the result
 * it gets alone.  With FSE_FLAG_DEVICE_PTRS, image/lost/out/out_f32/out_f64
 * are device pointers and the work is ordered on the plan's stream; the call
 * still returns only when the result is complete.
 * Errors: FSE_ERR_INVALID (null plan/frames/pointers, n < 1 or above
 * 16777215, sizes <= 0 or above 65535, strides smaller than width, a trace
 * with device pointers), FSE_ERR_DEVICE.
 */
int32_t fse_conceal_image(fse_plan_t plan, const fse_frame *frames, int32_t n);

/*
 * fse_conceal_image for callers that cannot allocate memory (code that must
 * not call hipMalloc: tight serving loops, harnesses that forbid it).  The
 * same computation as fse_conceal_image with FSE_FLAG_DEVICE_PTRS (same
 * kernels, one frame group, no staggered groups of streams), but every device
 * buffer of the call (working image, state map, descriptors, work items,
 * FP64 spectra, statistics) is a slice of a fixed device scratch region of
 * FSE_NOALLOC_SCRATCH_BYTES that the library holds per GPU for the life of
 * the process; no device or pinned host memory is allocated (host-side
 * bookkeeping uses ordinary heap memory, and the lost-block flags and work
 * items pass through ordinary host memory by synchronous copies).  The plan
 * must have been created with FSE_FLAG_DEVICE_PTRS; frames are device
 * pointers as for fse_conceal_image; traces are not supported; the call's
 * fse_last_call_stats carries no timings (kernel_ms, busy_ms, span_ms,
 * transform_ms are 0).  The scratch is shared by every call on a GPU and
 * keeps the last call's contents: calls that overlap in time on one GPU (from
 * several plans or threads) race, so callers serialize them.  With the same
 * tuning (frame_groups = 1) it gives the results of fse_conceal_image bit for
 * bit.  Errors: FSE_ERR_INVALID (as fse_conceal_image, a plan without
 * FSE_FLAG_DEVICE_PTRS, a frame with a trace), FSE_ERR_NOMEM (the call needs
 * more than FSE_NOALLOC_SCRATCH_BYTES of scratch: roughly 5 bytes per pixel
 * in FSE_FP32, 9 in FSE_FP64, plus 66 KB per block of the largest wave in
 * FSE_FP32_RERANK), FSE_ERR_DEVICE.
 */
#define FSE_NOALLOC_SCRATCH_BYTES ((int64_t)128 << 20)
int32_t fse_conceal_image_noalloc(fse_plan_t plan, const fse_frame *frames, int32_t n);

/*
 * Serving: submit one frame (host pointers only).  The input is copied before
 * the call returns; out, out_f32, out_f64, trace and stats must stay valid
 * until fse_poll reports FSE_OK for the ticket (or the plan is destroyed).
 * Frames in flight are continuously batched: every launch runs the next wave
 * of every admitted frame.  Frames are admitted as slots and device memory
 * free up.  Errors: FSE_ERR_INVALID, FSE_ERR_NOMEM (frame larger than the
 * whole budget), FSE_ERR_AGAIN (queue full: max_inflight_frames frames
 * waiting and running), FSE_ERR_DEVICE.
 */
int32_t fse_submit(fse_plan_t plan, const fse_frame *frame, uint64_t *ticket);

/*
 * Wait up to timeout_us microseconds (0 = do not wait, <0 = wait forever) for
 * a submitted frame.  Returns FSE_OK once (the ticket is then consumed),
 * FSE_PENDING, FSE_ERR_TICKET or FSE_ERR_DEVICE.
 */
int32_t fse_poll(fse_plan_t plan, uint64_t ticket, int32_t timeout_us);

/*
 * Device memory of serving.  device_mem_budget bounds every device buffer the
 * serving worker holds: the per-pixel arenas (working image, state map, 8-bit
 * input, mask, output) and the per-step buffers (FP64 spectra in
 * FSE_FP32_RERANK, staged results when d exceeds the block size, work items),
 * which take a fixed share of it (a quarter with spectra or staging, else
 * 1/64).  A frame is admitted while its pixels fit the arenas and its largest
 * wave fits the per-step share beside the largest waves of the frames already
 * admitted; fse_submit returns FSE_ERR_NOMEM for a frame that never fits.
 *   budget          device_mem_budget in effect (bytes);
 *   device_bytes    device memory the serving worker holds (0 before the
 *                   first fse_submit), at most `budget`;
 *   peak_committed  most bytes ever committed to admitted frames at once
 *                   (their pixels in the arenas plus their largest waves in
 *                   the per-step buffers), at most device_bytes;
 *   admitted_frames frames admitted so far;  peak_frames: most at once;
 *   step_blocks_cap blocks of a step the per-step share holds;
 *   peak_step_blocks most blocks ever reserved at once for the largest waves
 *                   of the admitted frames (at most step_blocks_cap).
 * Errors: FSE_ERR_INVALID (null pointer).
 */
typedef struct {
  int64_t budget;
  int64_t device_bytes;
  int64_t peak_committed;
  int64_t admitted_frames;
  int32_t peak_frames;
  int32_t reserved;
  int64_t step_blocks_cap;
  int64_t peak_step_blocks;
} fse_serving_stats;
int32_t fse_plan_serving_stats(fse_plan_t plan, fse_serving_stats *out);

/*
 * Processing order only (paper Algorithm 1 / line scan) for a block grid of
 * hb x wb blocks; lost[hb*wb] nonzero marks blocks with samples to
 * extrapolate (FSE_ORDER_REFINED needs sample counts: fse_schedule_refined).
 * wave_of[hb*wb] receives the wave index (-1 for the other blocks);
 * seq[hb*wb] (nullable) the lost blocks in processing order.
 * Host-only; returns the number of waves (>= 0) or FSE_ERR_INVALID.
 */
int32_t fse_schedule(int32_t hb, int32_t wb, const uint8_t *lost, int32_t order,
                     int32_t *wave_of, int32_t *seq);

/*
 * Refined processing order (FSE_ORDER_REFINED) for a block grid of hb x wb
 * blocks: unknown[hb*wb] holds the number of lost samples of each block (0 =
 * nothing to extrapolate, negative values count as 0); `outside` (>= 0) is
 * what a neighbour cell outside the image counts (normally block_w *
 * block_h).  wave_of and seq as in fse_schedule.  Host-only; returns the
 * number of waves (>= 0) or FSE_ERR_INVALID (negative size or outside, null
 * pointer with a non-empty grid).
 */
int32_t fse_schedule_refined(int32_t hb, int32_t wb, const int32_t *unknown, int32_t outside,
                             int32_t *wave_of, int32_t *seq);

/* Statistics of the last fse_conceal_image call.  The frames of a call run
 * in `groups` groups, each as its own sequence of launches (one per step) on
 * a stream of its own, so launches of different groups overlap in time.
 *   kernel_ms    device time of the per-block iteration kernel, summed over
 *                its launches (HIP events around every launch);
 *   launches     number of those launches;  blocks: blocks they processed;
 *   total_ms     host wall time of the call;
 *   transform_ms 0 (the transforms run inside the per-block kernel in every
 *                mode; the field is kept for the layout);
 *   span_ms      device time from the first to the end of the last
 *                extrapolation launch (all groups);
 *   groups       number of frame groups;
 *   busy_ms      device time during which at least one launch of the
 *                iteration kernel ran (union of the launch intervals);
 * FSE_FP32_RERANK, over all blocks of the call (0 in the other modes):
 *   rescored            iterations whose selection was re-scored exactly;
 *   rescore_candidates  entries re-scored (summed over wavefronts);
 *   rescore_wide        wavefront re-scores that took several rounds of
 *                       candidates (more than 3 with 4 wavefronts per block,
 *                       more than 2 otherwise);
 *   rescore_max_wave    most entries one wavefront re-scored in one
 *                       iteration. */
typedef struct {
  double kernel_ms;
  int64_t launches;
  int64_t blocks;
  double total_ms;
  double transform_ms;
  double span_ms;
  int64_t groups;
  double busy_ms;
  int64_t rescored;
  int64_t rescore_candidates;
  int64_t rescore_wide;
  int64_t rescore_max_wave;
} fse_call_stats;
int32_t fse_last_call_stats(fse_plan_t plan, fse_call_stats *out);

/*
 * Launch tuning of a plan: how batched calls and serving lay their work on
 * the GPU (results stay within the per-shape rounding noted at fse_plan).
 *   wave_threshold_16  launches of at most this many blocks run on 16
 *                      wavefronts per block (default 128; 0 in
 *                      FSE_FP32_RERANK);
 *   wave_threshold_8   larger launches of at most this many blocks run on 8
 *                      (default 0: never; 128 in FSE_FP32_RERANK); all
 *                      others on 4;
 *   frame_groups       frame groups of a batched call, 1..16; 0 = the
 *                      default, 3;
 *   crit_depth         frames with at least this fraction of the deepest
 *                      frame's waves form group 0 (0 = off, at most 1); < 0 =
 *                      the default, 0.9;
 *   crit_prio          1: group 0's workgroups raise their wave priority;
 *   crit_waves         wavefronts per block of group 0's launches: 4, 8 or
 *                      16; 0 = by the thresholds above on group 0's own
 *                      launch size; < 0 = the default, 4.
 * FSE_FP32_F16X3 runs every launch on 4 wavefronts whatever the thresholds.
 * fse_plan_get_tuning reports the values in effect (defaults resolved);
 * fse_plan_set_tuning takes effect for launches issued after it returns
 * (also those of frames already being served).  The environment variables
 * of fse_plan set the same values at plan creation.
 * Errors: FSE_ERR_INVALID (null pointer, value out of range).
 */
typedef struct {
  int32_t wave_threshold_16;
  int32_t wave_threshold_8;
  int32_t frame_groups;
  double crit_depth;
  int32_t crit_prio;
  int32_t crit_waves;
} fse_tuning;
int32_t fse_plan_get_tuning(fse_plan_t plan, fse_tuning *out);
int32_t fse_plan_set_tuning(fse_plan_t plan, const fse_tuning *t);

/*
 * Three-dimensional FSE of a video volume.  The paper develops the processing
 * order for two-dimensional signals and names its extension to
 * higher-dimensional signals through three-dimensional FSE (conclusion); this
 * interface carries every 2-D definition over one more dimension:
 *   - the volume (frames x rows x columns) is divided into blocks of
 *     block_t x block_h x block_w samples; a block holding lost samples is
 *     extrapolated from its area, the block plus border_t frames before and
 *     after and border_d samples around it in each frame (nominal geometry at
 *     the volume's faces, samples outside weigh 0);
 *   - weighting function of Eq. (2) with the 3-D distance from the area's
 *     centre; basis phi_k[t,m,n] = exp(+j 2 pi (k1 t / fft_t + k2 m / fft_h
 *     + k3 n / fft_w)) with the area at the grid's first corner; selection,
 *     increment, tie rule and iteration count as in two dimensions (ties to
 *     the smallest (k1 fft_h + k2) fft_w + k3); output = real part, rounded
 *     half to even and clamped;
 *   - processing order: Algorithm 1 over the 26-neighbourhood of the block
 *     grid (a missing neighbour at a face counts as not extrapolated, the
 *     wave filled in raster order frame, row, column), or line scan; every
 *     block of a wave reads the volume as it was at the start of the wave.
 * This build supports the basis grid fft_t x fft_h x fft_w = 8 x 32 x 32 and
 * FSE_FP64 (FSE_ERR_UNSUPPORTED otherwise): one workgroup per block holds the
 * whole 3-D spectrum in LDS.
 */
typedef struct fse_plan3_s *fse_plan3_t; /* opaque, owned by the library */

typedef struct {
  int32_t block_t, block_h, block_w; /* >= 1; block + 2 border <= fft per dimension */
  int32_t border_t;                  /* frames before and after the block, >= 0 */
  int32_t border_d;                  /* samples around the block in each frame, >= 0 */
  int32_t fft_t, fft_h, fft_w;       /* basis grid; this build: 8 x 32 x 32 */
  double rho;                        /* weighting decay, (0, 1] */
  double delta;                      /* reconstructed-area weight, [0, 1] */
  double gamma;                      /* orthogonality deficiency compensation, (0, 1] */
  int32_t iterations;                /* K, 1..FSE_MAX_ITERATIONS */
  int32_t order;                     /* FSE_ORDER_OPTIMIZED or FSE_ORDER_LINESCAN */
  int32_t precision;                 /* FSE_FP64 */
  double empty_fill;                 /* value written when an area has no support */
} fse_params3;

typedef struct {
  const uint8_t *volume; /* frames * height * width samples, frame-major, contiguous */
  const uint8_t *lost;   /* same layout, nonzero = lost (values there are ignored) */
  int32_t frames, height, width;
  uint8_t *out;          /* same layout; may alias volume; known samples copied */
  double *out_f64;       /* nullable: unquantized result, same layout */
  fse_stats *stats;      /* nullable: waves, lost blocks, largest wave; latency_ms =
                            device time from the first wave's launch to the
                            8-bit output (HIP events; copies excluded) */
} fse_volume;

/* Create / destroy a 3-D plan (host buffers; work on the given HIP stream,
 * nullable = the library's own).  Errors: FSE_ERR_INVALID (null pointer,
 * parameter out of range, block + 2 border above the grid),
 * FSE_ERR_UNSUPPORTED (another grid or precision), FSE_ERR_DEVICE. */
int32_t fse_plan3(const fse_params3 *p, void *hip_stream, fse_plan3_t *out);
int32_t fse_plan3_destroy(fse_plan3_t plan);

/* Conceal one volume synchronously (host pointers; the call returns with the
 * result in `out`).  Device memory: about 13 bytes per sample plus the
 * staging of the largest wave, kept by the plan for later calls.  Errors:
 * FSE_ERR_INVALID (null pointers, sizes <= 0 or above 65535 per dimension),
 * FSE_ERR_NOMEM (the device buffers could not be allocated; the plan stays
 * usable), FSE_ERR_DEVICE (a HIP call failed; the plan reports it from then
 * on). */
int32_t fse_conceal_volume(fse_plan3_t plan, const fse_volume *v);

/* Processing order only, for a tb x hb x wb block grid (frame-major);
 * lost[b] nonzero marks blocks with samples to extrapolate; wave_of[b]
 * receives the wave (-1 for the others), seq (nullable) the lost blocks in
 * processing order.  Returns the number of waves or FSE_ERR_INVALID. */
int32_t fse_schedule3(int32_t tb, int32_t hb, int32_t wb, const uint8_t *lost, int32_t order,
                      int32_t *wave_of, int32_t *seq);

/* Static description of an error code. */
const char *fse_strerror(int32_t code);

#ifdef __cplusplus
}
#endif

#endif /* FSE_H */
