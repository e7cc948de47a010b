/*
 * gmm.h - C ABI of the RGB-D mixture-of-Gaussians background segmentation library (gfx950).
 *
 * The library runs, per pixel and per frame, the adaptive Gaussian-mixture background model
 * of Sec. III.A of "GPU based GMM segmentation of Kinect data" (Amamra, Mouats, Aouf): M
 * Gaussians per pixel with means, variances and positive weights summing to one; a match test
 * against the components in decreasing w/sigma order; an online update of weights, means and
 * variances (with replacement of the least probable component on no match); selection of the
 * background components by the cumulative-weight threshold T; and classification of the pixel
 * as foreground when it fits no background component. Update rules the paper leaves to its
 * reference [6] (Stauffer and Grimson) follow that method. The colour image (uint8 RGB) and the
 * depth map (uint16 millimetres) are modelled separately (Sec. III.B) and their two binary
 * foreground images are fused by the counter rule of List 1 (Sec. III.C).
 *
 * Conventions for every entry point:
 *   - Every function returns a gmm_status. Arguments are validated synchronously, before any
 *     device work; on error nothing is enqueued and gmm_last_error() describes the problem.
 *     The library never aborts and never throws across this boundary.
 *   - Frame and mask pointers are DEVICE pointers owned by the caller. They must stay valid
 *     until the stream has executed the enqueued work.
 *   - `stream` is a hipStream_t (NULL = the device's null stream). Apply and fuse calls are
 *     asynchronous with respect to the host.
 *   - Foreground masks are bit-packed: ceil(width*height/64) uint64 words; word i holds pixels
 *     64i .. 64i+63 of the row-major frame, least significant bit first; pad bits are 0.
 *     Mask pointers must be 8-byte aligned.
 *   - A handle is not thread-safe; distinct handles are independent. Work on one handle must be
 *     ordered by the caller (one stream, or events), since every call reads and rewrites the
 *     handle's per-pixel state.
 *   - Execution faults surface at the caller's synchronisation; the handle's state is then
 *     unspecified.
 */
#ifndef RGBD_GMM_H
#define RGBD_GMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GMM_OK = 0,
  GMM_ERR_INVALID_ARG = -1,    /* argument outside its documented range or layout         */
  GMM_ERR_OUT_OF_MEMORY = -2,  /* a device or host allocation failed                      */
  GMM_ERR_DEVICE = -3,         /* a HIP runtime call or kernel launch failed              */
  GMM_ERR_STATE = -4,          /* the call does not apply to this handle (e.g. fuse on a
                                  single-modality handle)                                  */
  GMM_ERR_UNSUPPORTED = -5     /* a (M, state dtype) combination that is not compiled      */
} gmm_status;

/* modality bit mask */
enum { GMM_RGB = 1, GMM_DEPTH = 2 };
/* storage type of the per-pixel mixture state (arithmetic is always fp32) */
enum { GMM_F32 = 0, GMM_F16 = 1, GMM_BF16 = 2 };
/* which model the handle runs */
enum { GMM_SEPARATE = 0,       /* the method: colour and depth mixtures kept apart (Sec. III.B),
                                  their masks fused by List 1 (Sec. III.C)                   */
       GMM_AUGMENTED = 1 };    /* the alternative Sec. III.B describes and rejects: one mixture
                                  over four channels (R, G, B, D8), D8 = min(255, depth >> 4),
                                  the depth in 16 mm steps as a fourth intensity byte; one
                                  isotropic variance per component, colour sigma0 / var_min */
/* rate rho of the mean and variance updates */
enum { GMM_RHO_ALPHA = 0,      /* rho = alpha                                               */
       GMM_RHO_DENSITY = 1 };  /* rho = alpha * N(x | mu, var I): the matched component's
                                  isotropic Gaussian density at x before the update (the rate
                                  of the paper's reference [6], Stauffer and Grimson)         */
/* depth value 0 ("no reading" on a Kinect-class sensor) */
enum { GMM_HOLE_SKIP = 0,      /* state untouched, pixel classified background             */
       GMM_HOLE_AS_VALUE = 1 };/* 0 is treated as an ordinary distance                     */

/*
 * Model parameters (Sec. III.A): M Gaussians per pixel (the paper uses 3 <= M <= 5; 1 and 2
 * are accepted for closed-form tests), learning rate alpha (also the rate of the mean and
 * variance updates), match threshold k in standard deviations (strict: d^2 < k^2 sigma^2),
 * background weight threshold T. Index 0 of the two-element arrays is colour, 1 is depth.
 */
typedef struct {
  int32_t width, height;   /* > 0, width*height < 2^29 (32-bit byte offsets in the kernels) */
  int32_t modalities;      /* GMM_RGB, GMM_DEPTH or both                                    */
  int32_t M;               /* 1..5                                                          */
  float alpha;             /* (0, 1]                                                        */
  float k;                 /* > 0                                                           */
  float T;                 /* (0, 1)                                                        */
  float sigma0[2];         /* > 0: standard deviation of a newly created component          */
  float var_min[2];        /* 0 < var_min <= sigma0^2: floor of every variance              */
  float w_init;            /* (0, 1]: weight given to a new component before renormalising  */
  int32_t hole_policy;     /* GMM_HOLE_SKIP or GMM_HOLE_AS_VALUE                            */
  int32_t state_dtype;     /* GMM_F32, GMM_F16 or GMM_BF16                                  */
  int32_t device;          /* HIP device ordinal                                            */
  int32_t variant;         /* GMM_SEPARATE or GMM_AUGMENTED (needs both modalities)         */
  int32_t rho_mode;        /* GMM_RHO_ALPHA or GMM_RHO_DENSITY                              */
} gmm_config;

typedef struct gmm_handle gmm_handle;

/*
 * Fill `cfg` with this library's defaults for a width x height stream: alpha = 0.01, k = 2.5,
 * T = 0.7, sigma0 = {30, 50}, var_min = {(0.1 sigma0)^2} = {9, 25}, w_init = alpha,
 * GMM_HOLE_SKIP, GMM_F32, device 0, GMM_SEPARATE, GMM_RHO_ALPHA. The caller may then change
 * any field.
 */
gmm_status gmm_config_default(gmm_config* cfg, int32_t width, int32_t height, int32_t modalities,
                              int32_t M);

/*
 * Create a handle: validates `cfg`, allocates the per-pixel state on cfg->device and
 * initialises it synchronously - every component empty (w = 0, mu = 0, var = sigma0^2), and
 * for two-modality handles the fusion state of List 1 at I = 0, cpt = 0.
 * The handle owns all of its device memory. *out is set only on success. Each modality's state
 * must stay below 2 GiB (GMM_ERR_INVALID_ARG otherwise; fp32, M = 5: about 20 million pixels).
 */
gmm_status gmm_create(const gmm_config* cfg, gmm_handle** out);

/* Release a handle (synchronises the last stream it used first, then frees its state). NULL is a
 * no-op. */
gmm_status gmm_destroy(gmm_handle* h);

/*
 * Advance the model one frame and classify it (Sec. III.A, per modality; Sec. III.B keeps the
 * two modalities separate). GMM_ERR_STATE on a GMM_AUGMENTED handle.
 *   rgb        device HWC interleaved uint8 R,G,B; row y starts at rgb + y*rgb_pitch_bytes
 *              (pitch >= 3*width). NULL exactly when the handle has no colour modality.
 *   depth      device uint16 millimetres, row pitch depth_pitch_bytes (even, >= 2*width);
 *              NULL exactly when the handle has no depth modality.
 *   fg_rgb     device output mask of the colour model (see the mask layout above);
 *   fg_depth   device output mask of the depth model. Each is required for its modality and
 *              must be NULL for an absent one.
 * The fusion state of the handle is not touched (see gmm_fuse / gmm_apply_frame_fused).
 */
gmm_status gmm_apply_frame(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                           const uint16_t* depth, int64_t depth_pitch_bytes, uint64_t* fg_rgb,
                           uint64_t* fg_depth, void* stream);

/*
 * Fuse a colour and a depth foreground mask by List 1 (Sec. III.C), per pixel, updating the
 * handle's persistent fused bit I and counter cpt, and write the new I as the fused mask.
 * The depth foreground is taken as already registered to the colour frame (same size).
 * Requires a handle with both modalities, else GMM_ERR_STATE.
 */
gmm_status gmm_fuse(gmm_handle* h, const uint64_t* fg_rgb, const uint64_t* fg_depth,
                    uint64_t* fused, void* stream);

/*
 * The whole per-frame path in one launch: both mixture updates and List 1 fusion. Same
 * arguments as gmm_apply_frame plus the fused output mask. Bit-identical (masks and state) to
 * gmm_apply_frame followed by gmm_fuse. Requires both modalities, else GMM_ERR_STATE.
 */
gmm_status gmm_apply_frame_fused(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                                 const uint16_t* depth, int64_t depth_pitch_bytes,
                                 uint64_t* fg_rgb, uint64_t* fg_depth, uint64_t* fused,
                                 void* stream);

/*
 * The four-channel variant of Sec. III.B (a GMM_AUGMENTED handle, else GMM_ERR_STATE): one
 * mixture step per pixel on x = (R, G, B, min(255, depth >> 4)) and its foreground mask `fg`.
 * rgb, depth and their pitches as in gmm_apply_frame; all three pointers are required. With
 * GMM_HOLE_SKIP a depth of 0 leaves the pixel's state untouched and classifies it background.
 * A single-stream path for comparisons: batches and the serving executor reject such handles.
 */
gmm_status gmm_apply_frame_augmented(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                                     const uint16_t* depth, int64_t depth_pitch_bytes, uint64_t* fg,
                                     void* stream);

/* Text of the last error on the calling thread; valid until that thread's next call. */
const char* gmm_last_error(void);

/*
 * Measurement aid: when `wave_bytes` is a device array of ceil(width*height/64) uint64, every
 * later launch on this handle (plain or batched) ADDS to entry i the bytes of mixture state that
 * wave i (pixels 64i..64i+63) read and wrote. The traffic of a frame depends on the data: a
 * pixel that matches its top-ranked component and keeps it reads what decides that (the second
 * rank's variance, or in the fp32 form its stored key and the tile's scale) and writes only what
 * the step changed; any other pixel reads its whole state and writes the values that changed.
 * NULL stops recording. The caller owns (and zeroes) the array.
 * Batched launches copy the record pointer into their descriptors when these are prepared
 * (gmm_batch_set_frames; every gmm_batch_apply, gmm_batch_apply_static and executor tick), and a launch runs
 * the counting kernel only when one of its descriptors carries a record: a batched launch captured
 * into a graph before the slots were prepared with the record keeps the kernel that does not
 * count, so capture again after preparing them.
 */
gmm_status gmm_set_traffic_record(gmm_handle* h, uint64_t* wave_bytes);

/* Device bytes held by the handle's per-pixel state. */
gmm_status gmm_state_bytes(const gmm_handle* h, size_t* device_bytes);

/*
 * Number of doubles in the canonical state layout used by gmm_read_state / gmm_write_state:
 *   [colour block][depth block][I][cpt]
 * colour block: 5 x M x npix  parameters (muR, muG, muB, var, w), each rank-major;
 * depth block:  3 x M x npix  parameters (mu, var, w);
 * I and cpt:    npix each, present only for two-modality handles.
 * Blocks of absent modalities are omitted. A GMM_AUGMENTED handle has one block,
 * 6 x M x npix parameters (muR, muG, muB, muD8, var, w), and no I, cpt. Components appear in rank order (w/sigma
 * descending); an empty component has w = 0.
 */
gmm_status gmm_state_size(const gmm_handle* h, size_t* n_doubles);

/*
 * Copy the state out in the canonical layout (host memory, float64). Synchronises `stream`.
 * fp32 state keeps the weights of each 64-pixel tile as one scale times per-component scaled
 * weights (a frame's common decay of every weight goes into the scale alone); a depth pixel
 * that kept its state through k missing readings carries the factor (1/(1-alpha))^k besides.
 * The canonical weight is the fp32 product of scale and factor (as the kernels form it) times
 * the scaled weight, exact in float64. Every other value is copied exactly.
 */
gmm_status gmm_read_state(gmm_handle* h, double* host_out, void* stream);

/*
 * Replace the state from the canonical layout (host memory, float64), rounding each value to
 * the storage type to nearest, ties to even (fp32 weights are stored with scale 1 and no
 * missing-reading factor, so a read followed by a write can change the low bits of the
 * weights). I must be 0 or 1 and cpt in [-3, 3], else GMM_ERR_INVALID_ARG. Synchronises `stream`.
 */
gmm_status gmm_write_state(gmm_handle* h, const double* host_in, void* stream);

/*
 * Device-side snapshot of the state, for rolling a handle back (replaying the same frames from
 * the same state, trial launches): copies gmm_state_bytes bytes of the state, in the library's
 * own device layout, to (save) or from (restore) the caller's device buffer `device_dst` /
 * `device_src` (any alignment; owned by the caller; restore takes only a buffer a save of a
 * handle with the same configuration filled). Asynchronous on `stream`.
 */
gmm_status gmm_state_save(gmm_handle* h, void* device_dst, void* stream);
gmm_status gmm_state_restore(gmm_handle* h, const void* device_src, void* stream);

/* ---- batched path: many streams, one persistent launch per frame-set --------------------- */

typedef struct gmm_batch gmm_batch;

/* One stream's frame and masks in a batched call; the same rules as gmm_apply_frame (device
 * pointers, pitches, NULL for an absent modality). `fused` is optional: non-NULL (two-modality
 * streams only) runs List 1 for that stream in the same launch, like gmm_apply_frame_fused. */
typedef struct {
  const uint8_t* rgb;
  int64_t rgb_pitch_bytes;
  const uint16_t* depth;
  int64_t depth_pitch_bytes;
  uint64_t* fg_rgb;
  uint64_t* fg_depth;
  uint64_t* fused;
} gmm_stream_io;

/* Launch shape of the persistent kernel: threads per block (256 or 512), pixels per tile (a
 * multiple of block_threads, at most 64x it; a tile never spans two streams) and resident
 * blocks per compute unit (1..32; grid = blocks_per_cu x CU count, capped at the tile count). */
typedef struct {
  int32_t block_threads;
  int32_t tile_pixels;
  int32_t blocks_per_cu;
} gmm_batch_tuning;

/*
 * Group existing handles (same device, same M, same state dtype; each at most once) so that one
 * launch advances all of them by one frame. Uneven resolutions and modality mixes are allowed.
 * `n_slots` descriptor slots (1..4096) hold prepared frame-sets, so launches can be captured in
 * a hipGraph and replayed. The handles must outlive the batch and must not be used by other
 * calls while batch work on them is in flight. Default tuning: {256, 1024, 8}.
 * GMM_ERR_UNSUPPORTED for a GMM_AUGMENTED handle.
 */
gmm_status gmm_batch_create(gmm_handle* const* handles, int32_t n, int32_t n_slots, gmm_batch** out);

/* Release a batch (synchronises its last stream first); the handles stay valid. NULL: no-op. */
gmm_status gmm_batch_destroy(gmm_batch* b);

/* Set / query the launch shape. Setting it synchronises the batch's last stream and invalidates
 * graphs captured with the previous shape. */
gmm_status gmm_batch_set_tuning(gmm_batch* b, const gmm_batch_tuning* t);
gmm_status gmm_batch_get_tuning(const gmm_batch* b, gmm_batch_tuning* t);

/*
 * Prepare descriptor slot `slot` with one gmm_stream_io per handle (host array, in the order of
 * gmm_batch_create). Every stream is validated first; on error nothing changes. The descriptors
 * are uploaded asynchronously on `stream`; the host array may be reused when the call returns.
 */
gmm_status gmm_batch_set_frames(gmm_batch* b, int32_t slot, const gmm_stream_io* io, void* stream);

/*
 * Advance every stream of the batch one frame using the frames and masks of slot `slot`, in one
 * persistent launch on `stream`. Per stream, results (masks and state) are bit-identical to
 * gmm_apply_frame (or gmm_apply_frame_fused when `fused` was given). Allocates nothing and does
 * not synchronise: safe to capture in a hipGraph.
 */
gmm_status gmm_batch_run(gmm_batch* b, int32_t slot, void* stream);

/* gmm_batch_set_frames(b, 0, io, stream) followed by gmm_batch_run(b, 0, stream). */
gmm_status gmm_batch_apply(gmm_batch* b, const gmm_stream_io* io, void* stream);

/*
 * Choose the launch shape by timing trial launches over block_threads {256, 512} x tile
 * multiples {1, 2, 4, 8, 16} x blocks_per_cu {2, 4, 8, 16}, keep the fastest, and cache it for
 * this process per (device, M, state dtype, multiset of stream shapes and modalities). Each
 * candidate runs slot `slot` and up to three more prepared slots after it, in order, from the
 * same saved state. Every stream's state is restored afterwards (the slots' masks are
 * overwritten by the trials). Synchronous. Reports the winner and its time per launch.
 */
gmm_status gmm_batch_autotune(gmm_batch* b, int32_t slot, void* stream, gmm_batch_tuning* best,
                              double* best_ms);

/* Number of tiles of one launch under the current tuning. */
gmm_status gmm_batch_tiles(const gmm_batch* b, uint32_t* n_tiles);

/* ---- batched launch without allocation ---------------------------------------------------- */

#define GMM_STATIC_MAX_STREAMS 1024

/*
 * For callers that cannot allocate device memory - code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc: gmm_batch_apply for `n` existing handles (1 ..
 * GMM_STATIC_MAX_STREAMS; same device, M and state dtype; each at most once) without a
 * gmm_batch object. `io` is a host array of n stream entries (rules of gmm_batch_set_frames);
 * `tuning` is the launch shape (NULL: {256, 1024, 8}; limits of gmm_batch_tuning). Per stream,
 * masks and state are bit-identical to gmm_batch_apply (and so to gmm_apply_frame /
 * gmm_apply_frame_fused).
 * The per-call tables (stream descriptors and first tiles, about 212 KB at the maximum) live in
 * one static device array of the library, one per device, held until the process ends; the call
 * allocates no memory on the device or through any allocating library routine, and copies
 * nothing from host memory (the descriptors travel as kernel arguments), so it can be captured.
 * Every call on a device reuses that device's array, which keeps the last call's contents:
 * calls that overlap on one device (different streams, or threads without ordering) race and
 * must be ordered by the caller. More than GMM_STATIC_MAX_STREAMS streams: GMM_ERR_INVALID_ARG
 * before any device work. GMM_ERR_UNSUPPORTED for a GMM_AUGMENTED handle. Asynchronous on
 * `stream`.
 */
gmm_status gmm_batch_apply_static(gmm_handle* const* handles, int32_t n, const gmm_stream_io* io,
                                  const gmm_batch_tuning* tuning, void* stream);

/* ---- serving executor: ticks of host frames through one batched launch each --------------- */

typedef struct gmm_exec gmm_exec;

/* One stream's frame in a tick. Frames are read from host memory with dense rows (pitch
 * 3*width for colour, 2*width for depth) by DMA; masks are written to host memory. Host buffers
 * should be page-locked (hipHostMalloc, pinned torch tensors) for the copies to overlap device
 * work; they must stay valid and untouched until the tick completes (gmm_exec_poll). A NULL
 * mask pointer skips copying that mask back; non-NULL host_fused runs List 1 for the stream
 * (two-modality streams only). */
typedef struct {
  gmm_handle* handle;
  const uint8_t* host_rgb;
  const uint16_t* host_depth;
  uint64_t* host_fg_rgb;
  uint64_t* host_fg_depth;
  uint64_t* host_fused;
} gmm_exec_item;

/*
 * Executor for the serving loop: default-priority HIP streams (four copy-in, compute, copy-out)
 * pipeline consecutive ticks as in the paper's overlap of host transfers with device work
 * (Sec. IV, Fig. 4(a)); `ring` (1..64) bounds the ticks in flight. A completion thread records
 * each tick's completion time on the gmm_exec_now() clock.
 */
gmm_status gmm_exec_create(int32_t device, int32_t ring, gmm_exec** out);
/* Wait for all ticks, then release. NULL is a no-op. Attached handles stay valid. */
gmm_status gmm_exec_destroy(gmm_exec* x);
/* Launch shape of the batched kernel (same meaning and limits as gmm_batch_tuning). */
gmm_status gmm_exec_set_tuning(gmm_exec* x, const gmm_batch_tuning* t);
/* Give a stream two device frame slots, used by its frames in turn so that one frame can be
 * copied in while the previous one computes (all streams of an executor share M and the state
 * dtype). Reports the device bytes this adds, for memory admission.
 * GMM_ERR_UNSUPPORTED for a GMM_AUGMENTED handle (also in the two calls below). */
gmm_status gmm_exec_attach(gmm_exec* x, gmm_handle* h, size_t* device_bytes);
/* Release a stream's frame slots after its last tick has completed (waits for it). */
gmm_status gmm_exec_detach(gmm_exec* x, gmm_handle* h);
/* Device bytes of a stream created by gmm_exec_create_stream: its state (as gmm_state_bytes)
 * rounded up to 256 bytes, then its two frame slots. */
gmm_status gmm_exec_stream_bytes(const gmm_config* cfg, size_t* bytes);
/*
 * Create and attach a stream whose state and frame slots live in caller-provided device memory
 * `mem` (256-byte aligned, at least gmm_exec_stream_bytes). The state is initialised on the
 * executor's compute stream, ordered before every later tick: no allocation and no host
 * synchronisation, so streams can join a running server without stalling it. The caller keeps
 * `mem` until gmm_exec_destroy_stream.
 */
gmm_status gmm_exec_create_stream(gmm_exec* x, const gmm_config* cfg, void* mem, size_t bytes,
                                  gmm_handle** out);
/* Detach and release a stream made by gmm_exec_create_stream once its last tick has completed
 * (waits for that tick only); frees no device memory. */
gmm_status gmm_exec_destroy_stream(gmm_exec* x, gmm_handle* h);
/*
 * Advance the given streams (each at most once, none with two frames still in flight) by one
 * frame in one tick; returns at once with the tick's id (ids increase by 1 from 1). A stream's
 * frames are applied in launch order. Blocks only when `ring` ticks are already in flight. Per
 * stream, masks and state are bit-identical to gmm_apply_frame / gmm_apply_frame_fused on the
 * same frames.
 */
gmm_status gmm_exec_launch(gmm_exec* x, const gmm_exec_item* items, int32_t n, uint64_t* tick_id);
/* Completed ticks since the last poll, in launch order: ids and completion times (at most cap). */
gmm_status gmm_exec_poll(gmm_exec* x, uint64_t* tick_ids, double* t_done, int32_t cap, int32_t* n);
/* Block until every launched tick has completed. */
gmm_status gmm_exec_drain(gmm_exec* x);
/* The executor clock: seconds on a monotonic clock. */
double gmm_exec_now(void);

/* ---- evaluation ------------------------------------------------------------------------- */

/*
 * Confusion counts of a predicted foreground mask against a reference mask, the quantities
 * recall, precision and F1 are computed from (Sec. V.A, Eqs. 1-3): counts[0..3] = TP, FP, TN,
 * FN over the first npix pixels (pad bits ignored). pred, truth: device bit-packed masks in the
 * layout above; counts: device array of 4 uint64, overwritten (not accumulated). Asynchronous
 * on `stream`; no allocation.
 */
gmm_status gmm_mask_confusion(const uint64_t* pred, const uint64_t* truth, int64_t npix, uint64_t* counts,
                              void* stream);

/*
 * Measurement aid: copy `bytes` bytes from device `src` to device `dst` (both 16-byte aligned,
 * not overlapping) with the library's streaming copy kernel, asynchronously on `stream`. It reads
 * and writes exactly `bytes` each, which makes it the yardstick of the memory system's practical
 * read+write rate beside the mixture kernels and the calibration of the HBM traffic counters.
 * No allocation.
 */
gmm_status gmm_device_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Library version as major*10000 + minor*100 + patch. */
int32_t gmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RGBD_GMM_H */
