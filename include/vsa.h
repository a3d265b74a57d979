/*
 * vsa.h -- C ABI of libvsa, the MI355X (gfx950) per-frame video measure engine.
 *
 * The engine computes, on the GPU, the measures of Fassold's unified
 * shot-boundary / sampling-structure / dynamic-keyframe detector
 * (arXiv 2502.09202, Sec. III) and the cheap decisions on top of them:
 *
 *   - a luma pyramid (2x2 rounding box filter, per level) with the upper and
 *     lower fields (even / odd rows) of every frame (Sec. III.C);
 *   - an 8x8-block integer motion field by exhaustive SAD search in +-8
 *     working pixels (stands in for the dense optical flow of Sec. III.A);
 *   - the exact integer moments of the reference against the motion-
 *     compensated (warped) image, NCC, SWR = 1 - NCC, AMM (average motion
 *     magnitude) and ACT (geometric average of AMM and SWR) (Sec. III.A);
 *   - ACT of consecutive frames always; field measures v0, v1, v2 and the
 *     deep-check pairs only when the decision logic asks for them (the
 *     sparse, selective schedule of Sec. III.A), compacted on the device;
 *   - hardcut / dissolve (fast + deep check, Sec. III.B), progressive /
 *     interlaced TFF / BFF / 3:2 pulldown per shot (Sec. III.C), dynamic
 *     keyframes (Sec. III.D).
 *
 * Model: open streams (one per video), push one luma plane per stream, call
 * vsa_step() to process one time step of every stream that has a frame (or is
 * draining after vsa_stream_end), vsa_sync(), then poll per-frame and per-shot
 * records.  Records come out in frame order, a bounded number of frames after
 * the frame was pushed (the deep check looks ahead up to k_max+1 frames); a
 * shot record is final only once the next boundary (or the end) is known.
 * For one clip whose frames are all at hand, the offline form (vsa_clip_*)
 * gives the same records for the whole clip in one call, taking it a chunk
 * of frames per launch.
 *
 * Conventions
 *   - Every call that can fail returns a vsa_status (0 = VSA_OK, < 0 error);
 *     no C++ exception crosses this boundary.  vsa_last_error() describes the
 *     last failure of the calling thread.
 *   - The engine owns all device memory it allocates.  The caller owns every
 *     buffer it passes in (frames, output arrays) unless a call says otherwise.
 *   - Calls on one engine are serialised by an internal mutex; distinct
 *     engines are independent.
 *   - Pixel formats: 8-bit luma in uint8, or 10-bit luma in uint16 (values
 *     <= 1023, little endian).  Only the Y plane is read.  A 10-bit plane the
 *     library reads from host memory with a copy (VSA_SRC_HOST) is checked
 *     and refused with VSA_E_INVAL if a sample exceeds 1023; planes read in
 *     place (device memory, VSA_SRC_HOST_BORROW) are not checked, and such
 *     samples give unspecified measures (never an access outside the
 *     library's buffers).
 */
#ifndef VSA_H
#define VSA_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define VSA_ABI_VERSION 3

typedef int32_t vsa_status;
enum {
    VSA_OK = 0,
    VSA_E_INVAL = -1,        /* invalid argument (NULL, size, bit depth, pitch, ...)   */
    VSA_E_NOMEM = -2,        /* device or host allocation failed                        */
    VSA_E_ADMIT = -3,        /* stream refused: HBM budget or stream slots exhausted    */
    VSA_E_STATE = -4,        /* call not valid in the stream's state (push after end)   */
    VSA_E_DEVICE = -5,       /* HIP runtime error (the engine should be destroyed)     */
    VSA_E_AGAIN = -6,        /* stream already holds a frame waiting for a step         */
    VSA_E_UNSUPPORTED = -7   /* parameters outside what the kernels implement           */
};

/* Algorithm constants (the paper prints none).  Same meaning as the fields of
 * the JSON parameter file shipped with the package. */
typedef struct {
    int32_t block;        /* block edge; must be 8                                         */
    int32_t radius;       /* search radius R in working pixels; must be 8                   */
    int32_t wmax;         /* working level L = first pyramid level with width <= wmax        */
    int32_t lf_offset;    /* field level Lf = max(0, L - lf_offset); must be 1               */
    int32_t k_max;        /* default longest transition tested by the deep check (1..15)     */
    int32_t a_static_fx;  /* pair is STATIC if A < a_static_fx * B (A in 1/256 px)           */
    int32_t w_hist;       /* fast-check history length (1..16)                               */
    int32_t n_ss;         /* frames analysed per shot for sampling structure                 */
    double a0;            /* ACT = sqrt((AMM + a0) * SWR)                                    */
    double rho_f, theta_f;/* fast check fires if ACT > rho_f * mean(history) + theta_f       */
    double theta_f0;      /* ... or, with no history in the shot yet, if ACT > theta_f0      */
    double rho_d, theta_d;/* deep check verifies K if F_K > rho_d * P_K + theta_d            */
    double gamma;         /* transition length: first K with F_K - P_K >= gamma * max of them  */
    double tau_c;         /* interlace vote: frame combed if v0 > tau_c * min(v1, v2)         */
    double eps;           /* progressive if combed <= eps n, interlaced if >= (1 - eps) n     */
    double tau_p;         /* 3:2 pulldown if the mean v0 at two neighbouring positions of the
                             5-frame unit exceeds tau_p times the mean at each other one     */
    double theta_kf;      /* keyframe when accumulated ACT exceeds theta_kf                  */
    int32_t search;       /* motion field of frame pairs (Sec. III.A): 0 full search over
                             [-R, R]^2; 1 coarse-to-fine: full search on the 2x2-box image one
                             level coarser, then +-refine around twice that vector (reach
                             2R + refine).  Field pairs always take the full search.
                             2 dense inverse search flow for every pair, frame and field
                             pairs alike (the measure of vsa_flow_pair); the frame records
                             then carry n_pix = the plane's pixels and zero moments,
                             amm_num and n_blocks, and vsa_get_motion has no block field.   */
    int32_t refine;       /* refinement radius of the coarse-to-fine search; must be 1       */
} vsa_params;

typedef struct {
    int32_t device;            /* HIP device ordinal                                        */
    int32_t max_streams;       /* stream slots (1..1024)                                    */
    uint64_t hbm_budget_bytes; /* admission budget; 0 = 90% of free device memory at create */
    int32_t schedule;          /* VSA_SCHEDULE_SPARSE (the paper's) or VSA_SCHEDULE_DENSE   */
    int32_t use_graph;         /* must be 0: a captured HIP graph of a step costs more host
                                  time per replay than its direct launches (VSA_E_UNSUPPORTED) */
    const vsa_params* params;  /* NULL = built-in defaults (vsa_default_params)             */
    int32_t debug_log;         /* 1: keep a log of every sparse measure computed            */
    int32_t me_wgs_per_cu;     /* persistent motion-search workgroups per compute unit:
                                  0 = autotuned per step size, else 1..8 (results do not
                                  depend on it)                                              */
    int32_t profile;           /* time kernel launches with HIP events (see
                                  vsa_engine_kernel_times): 1 pyramid and motion search,
                                  2 every kernel and the whole step; 0 off                   */
    int32_t no_intensity;      /* 1: skip the unary intensity measure H(t) (Sec. III.A; no
                                  decision uses it): h_mean/h_std/h_mad are NaN and
                                  vsa_get_histogram fails with VSA_E_STATE; 0: computed      */
    int32_t profile_every;     /* with profile: time the launches of one step in this many
                                  (0 or 1: every step); timing events cost device time      */
    const char* params_json;   /* non-NULL: the parameters as a JSON object of the fields of
                                  vsa_params (vsa_params_from_json), used instead of params  */
    const char* autotune_cache;/* non-NULL: a text file of the launch tuner's choices, one per
                                  (compute units, search, step size bucket); read at create
                                  (a bucket found there is not tuned again) and appended as
                                  buckets settle.  Missing or unreadable: tuned as without   */
} vsa_engine_config;

enum { VSA_SCHEDULE_SPARSE = 0, VSA_SCHEDULE_DENSE = 1 };

typedef struct {
    int32_t width, height;     /* full-resolution luma size                                 */
    int32_t bit_depth;         /* 8 or 10                                                   */
    int32_t fps_num, fps_den;  /* nominal frame rate (informational)                        */
    int32_t k_max;             /* 0 = params default, else 1..15                            */
} vsa_stream_desc;

/* Where vsa_stream_push reads the plane from. */
enum {
    VSA_SRC_HOST = 0,          /* host memory; copied into engine-owned pinned memory before the
                                  call returns; the caller may reuse the buffer at once          */
    VSA_SRC_DEVICE_COPY = 1,   /* device memory; copied into engine-owned device memory before
                                  the call returns                                               */
    VSA_SRC_DEVICE_BORROW = 2, /* device memory read in place by the next vsa_step; the caller
                                  keeps it valid and unmodified until that step has completed:
                                  vsa_sync has returned, or vsa_collect counts it as published  */
    VSA_SRC_HOST_BORROW = 3    /* host memory (pinned by the caller, e.g. hipHostMalloc, for a
                                  direct DMA) uploaded by the next vsa_step without a host-side
                                  copy; kept valid and unmodified until that step has completed,
                                  as for VSA_SRC_DEVICE_BORROW                                   */
};

/* Per-frame record.  The pair measures describe (frame -> frame+1) at the
 * working level; v0..v2 are NaN unless field_mask says they were computed. */
typedef struct {
    int64_t frame, pts;
    int32_t flags;             /* VSA_F_* bits                                              */
    int32_t shot_id;           /* -1 for frames inside a transition                         */
    int32_t boundary;          /* 0 none, 1 hardcut, 2 dissolve: set on the first frame of a shot */
    int32_t boundary_k;        /* K* of that boundary (1 for a hardcut)                     */
    double ncc, swr, amm, act;
    int64_t mom[5];            /* Sx, Sy, Sxx, Syy, Sxy over the covered pixels             */
    int64_t n_pix, amm_num;    /* N = 64 B and A = sum over blocks of floor(256 |d|)        */
    int32_t n_blocks;
    uint32_t field_mask;
    double v[3];               /* v0 = ACT(U_t, D_t), v1 = ACT(U_t, D_t+1), v2 = ACT(D_t, U_t+1) */
    double h_mean, h_std, h_mad; /* Sec. III.A unary measure H(t) over the working-level image:
                                  mean, standard deviation (population) and mean absolute
                                  deviation about the mean of its intensity histogram      */
} vsa_frame_result;

enum {
    VSA_F_HAS_PAIR = 1, VSA_F_STATIC = 2, VSA_F_FAST_FIRED = 4, VSA_F_IN_TRANSITION = 8,
    VSA_F_KEYFRAME = 16, VSA_F_SHOT_START = 32, VSA_F_ANALYZED = 64
};

enum { VSA_SAMPLING_UNDETERMINED = 0, VSA_SAMPLING_PROGRESSIVE = 1, VSA_SAMPLING_TFF = 2,
       VSA_SAMPLING_BFF = 3, VSA_SAMPLING_PULLDOWN32 = 4 };

typedef struct {
    int32_t shot_id, pad0;
    int64_t first, last;
    int32_t in_boundary, in_k;
    int32_t sampling;          /* VSA_SAMPLING_*                                            */
    int32_t pulldown_phase;    /* position (mod 5, from the shot start) of the first mixed frame; -1 */
    int32_t n_analyzed, final_;
} vsa_shot_result;

typedef struct vsa_engine vsa_engine;

/* ABI version of the loaded library (VSA_ABI_VERSION). */
int32_t vsa_abi_version(void);

/* Fill *out with the built-in parameter defaults. */
void vsa_default_params(vsa_params* out);

/* The parameters from a JSON object whose keys are vsa_params' field names
 * (integers for the int32 fields, numbers for the doubles); fields it does
 * not name keep their defaults.  VSA_E_INVAL (out unchanged) for a syntax
 * error, an unknown key, a non-integer int32 field or a value out of int32
 * range.  The package's params/default.json is such an object. */
vsa_status vsa_params_from_json(const char* json, vsa_params* out);

/* Create an engine on cfg->device; allocates the engine-wide device buffers.
 * Errors: VSA_E_INVAL (NULL, bad sizes), VSA_E_UNSUPPORTED (params the kernels
 * do not implement), VSA_E_DEVICE, VSA_E_NOMEM. */
vsa_status vsa_engine_create(const vsa_engine_config* cfg, vsa_engine** out);

/* Wait for queued work, close every stream and free all device memory.
 * NULL is a no-op. */
void vsa_engine_destroy(vsa_engine* e);

/* HBM bytes a stream of this shape holds while open (used for admission);
 * 0 if the description is invalid. */
uint64_t vsa_stream_footprint(const vsa_engine* e, const vsa_stream_desc* d);

/* Open a stream: one video analysed by the method of Sec. III, with its own
 * pyramid ring, measure history and decision state in device memory.  *sid
 * receives the stream id.  Frames smaller than a 2 x 2 grid of blocks at the
 * working level give VSA_E_INVAL; no free slot or not enough budget gives
 * VSA_E_ADMIT (admission by HBM budget). */
vsa_status vsa_stream_open(vsa_engine* e, const vsa_stream_desc* d, int32_t* sid);

/* Hand over the next frame of stream sid: its luma plane only (the measures
 * of Sec. III.A work on intensity), W x H samples with rows pitch_bytes apart,
 * read from host or device memory as `src` says (VSA_SRC_*; ownership there).
 * pts is carried into the frame's record.  VSA_E_AGAIN if the previous frame
 * has not been taken by a vsa_step yet; VSA_E_STATE after vsa_stream_end;
 * VSA_E_INVAL for a NULL plane or a pitch below one row. */
vsa_status vsa_stream_push(vsa_engine* e, int32_t sid, const void* luma, int64_t pitch_bytes,
                           int32_t src, int64_t pts);

/* Push one plane to each of n streams in one call (same rules as
 * vsa_stream_push for each).  status (nullable) receives the n individual
 * results; the call returns VSA_OK if all succeeded, else the first error. */
vsa_status vsa_stream_push_batch(vsa_engine* e, int32_t n, const int32_t* sids, const void* const* planes,
                                 const int64_t* pitches, int32_t src, const int64_t* pts, int32_t* status);

/* End of stream: later steps drain the look-ahead and close the last shot. */
vsa_status vsa_stream_end(vsa_engine* e, int32_t sid);

/* 1 once every record of an ended stream has been published (by vsa_sync or
 * vsa_collect), 0 if not, < 0 on error. */
int32_t vsa_stream_done(vsa_engine* e, int32_t sid);

/* Enqueue one time step over every open stream: the pyramid and fields of
 * each new frame (Sec. III.C), the consecutive pair's motion field and
 * measures (Sec. III.A), the sparse pairs the decision logic requested in the
 * previous step (fields Sec. III.C, deep check Sec. III.B), and one advance of
 * each stream's sequential pass (Sec. III.B-D).  Asynchronous.  hip_stream
 * (nullable) is a hipStream_t: the step starts after the work already queued
 * on it and work queued on it later starts after the step.  Errors:
 * VSA_E_INVAL, VSA_E_DEVICE. */
vsa_status vsa_step(vsa_engine* e, void* hip_stream);

/* Wait for every queued step and publish its records to the host queues.
 * Errors: VSA_E_INVAL, VSA_E_DEVICE. */
vsa_status vsa_sync(vsa_engine* e);

/* Publish, without waiting, the records of every step the device has already
 * completed (each step snapshots the output cursors after its decisions), so
 * that vsa_poll_* return them; the non-blocking form of vsa_sync for serving
 * loops.  *steps_published (nullable) receives the number of steps, counted
 * from the engine's first, whose records are published.  Errors:
 * VSA_E_INVAL, VSA_E_DEVICE. */
vsa_status vsa_collect(vsa_engine* e, int64_t* steps_published);

/* Copy up to cap published per-frame records of stream sid into out (the
 * caller's array), in frame order, and remove them from the queue: the
 * frame's pair measures (Sec. III.A), field measures when computed
 * (Sec. III.C) and its labels: boundary, transition, shot, keyframe
 * (Sec. III.B, III.D).  Returns the number copied, or < 0 on error. */
int32_t vsa_poll_frames(vsa_engine* e, int32_t sid, vsa_frame_result* out, int32_t cap);

/* Same for per-shot records: each shot between two boundaries (Sec. III.B)
 * with its sampling structure, field order and pulldown phase (Sec. III.C);
 * a shot is reported once the next boundary or the end is known. */
int32_t vsa_poll_shots(vsa_engine* e, int32_t sid, vsa_shot_result* out, int32_t cap);

/* Per-frame records of every stream in one call (serving interface, not in
 * the paper): up to cap records, each stream's in frame order, with sids[i]
 * the stream of out[i]; both arrays are the caller's.  Returns the number
 * copied, or < 0 on error. */
int32_t vsa_poll_frames_all(vsa_engine* e, int32_t* sids, vsa_frame_result* out, int32_t cap);

/* Motion field (Sec. III.A; here 8x8 block matching) of the pair
 * (frame -> frame+1) of stream sid at the working level, as nby x nbx pairs
 * (dx, dy) of int8 written to mv_xy (cap_blocks pairs, the caller's array;
 * NULL to query nbx, nby), if that frame is still held on the device (the
 * last 2 k_max + 7 frames).  Synchronises the engine.  VSA_E_INVAL otherwise;
 * VSA_E_UNSUPPORTED for an engine with the dense flow (search 2). */
vsa_status vsa_get_motion(vsa_engine* e, int32_t sid, int64_t frame, int8_t* mv_xy,
                          int32_t cap_blocks, int32_t* nbx, int32_t* nby);

/* Sec. III.A: the intensity histogram H(t) of frame `frame` over its
 * working-level image: bins[v] = pixels with value v, v < 2^bit_depth (the
 * frame's h_mean, h_std and h_mad are taken from it).  Held for the last rs
 * frames stepped (the stream's ring).  *nbins (if not NULL) receives
 * 2^bit_depth; with bins NULL only that count is returned.  The caller owns
 * bins (cap entries).  Waits for the engine's queued work.  VSA_E_INVAL: no
 * such stream, cap < 2^bit_depth, or the frame is not held on the device;
 * VSA_E_STATE: the engine was created with no_intensity. */
vsa_status vsa_get_histogram(vsa_engine* e, int32_t sid, int64_t frame, uint32_t* bins, int32_t cap,
                             int32_t* nbins);

/* Free the slot at once, without waiting for the device: records not yet
 * polled are dropped, and the stream's device memory is reused only after the
 * queued steps that read it have completed. */
vsa_status vsa_stream_close(vsa_engine* e, int32_t sid);

/* Instrumentation (not in the paper).  Engine counters, the first n of: [0] steps, [1] streams open, [2] streams
 * admitted, [3] admissions refused, [4] HBM bytes held by streams, [5] budget
 * bytes, [6] sparse pair tasks planned, [7] consecutive pair tasks run,
 * [8] blocks of the consecutive pairs, [9] blocks of the sparse pairs
 * (device-side figures as of the last vsa_sync), and host nanoseconds spent
 * in vsa_step: [10] building step descriptors, [11] uploads, [12] kernel
 * launches and stream ordering, [13] in total. */
vsa_status vsa_engine_counters(vsa_engine* e, uint64_t* out, int32_t n);

/* Instrumentation (not in the paper).  State of the motion-search launch
 * autotuner for size bucket `bucket` (0..31, floor(log2) of a step's
 * consecutive-pair tiles): *best is the chosen candidate, or -1 while the
 * bucket is being tuned (or pinned by me_wgs_per_cu).  For the first min(cap,
 * count) candidates, wgs[2c], wgs[2c+1] are its workgroups per CU of the
 * consecutive and the sparse grid, windows[c] its finished timing windows and
 * step_ms[c] the step period of its fastest window (0 without any).  Any of the
 * arrays may be NULL when cap is 0.  Returns the candidate count, or a
 * negative vsa_status (bad engine or bucket, or cap < 0). */
int32_t vsa_engine_tuning(vsa_engine* e, int32_t bucket, int32_t* best, int32_t* wgs, int32_t* windows,
                          double* step_ms, int32_t cap);

/* Accumulated device time per kernel of engines created with profile = 1
 * (slots 0-3) or 2 (all), measured with HIP events on the stream each runs
 * on, for the steps completed by the last vsa_sync: ms[i] total milliseconds
 * and launches[i] launch count of i = 0 pyramid (K1), 1 motion search of the
 * consecutive pairs, 8-bit, 2 the same, 10-bit, 3 motion search of the
 * sparse pairs (both depths), 4 decisions (K6), 5 whole step (descriptor
 * upload to end of K6).  Either pointer may be NULL; reset = 1 clears the
 * totals. */
vsa_status vsa_engine_kernel_times(vsa_engine* e, double* ms, uint64_t* launches, int32_t reset);

/* ---- offline form: one whole clip, look-ahead batched --------------------- */

/* The same analysis as a stream of the engine (Sec. III: identical records and
 * shots), for one clip whose frames are all at hand.  Instead of one frame per
 * step, `chunk` frames at a time go through the pyramid and the consecutive
 * pairs' motion search in one launch each; the sequential pass (Sec. III.B-D)
 * then runs over them, with rounds of sparse pairs (Sec. III.A's selective
 * schedule) wherever it asks for measures, before the next chunk.  A lone
 * clip thus fills the GPU without other streams beside it. */
typedef struct vsa_clip vsa_clip;

typedef struct {
    int32_t device;            /* HIP device ordinal                                        */
    int32_t width, height;     /* full-resolution luma size of every frame                  */
    int32_t bit_depth;         /* 8 or 10                                                   */
    int32_t k_max;             /* 0 = params default, else 1..15                            */
    int32_t chunk;             /* frames per chunk, 1..4096; 0 = 256 (the first chunk takes
                                  min(chunk, max(16, chunk / 4)) frames, so that decisions
                                  start early).  Device memory grows with it (a ring of
                                  2 chunk + 2 k_max + 8 frame slots)                        */
    int32_t schedule;          /* VSA_SCHEDULE_SPARSE (the paper's) or VSA_SCHEDULE_DENSE   */
    int32_t no_intensity;      /* 1: skip H(t) (h_mean/h_std/h_mad are NaN)                 */
    int32_t me_wgs_per_cu;     /* persistent motion-search workgroups per CU, 0 = default   */
    const vsa_params* params;  /* NULL = built-in defaults                                  */
    int32_t debug_log;         /* 1: keep a log of the sparse measures the sequential pass
                                  requests (vsa_clip_debug_log)                              */
} vsa_clip_config;

/* Create a clip analyser on cfg->device and allocate its device memory (sized
 * by frame size, k_max and chunk).  Errors as vsa_engine_create, and
 * VSA_E_INVAL for a frame smaller than a 2 x 2 grid of blocks at the working
 * level or a chunk outside 1..4096. */
vsa_status vsa_clip_create(const vsa_clip_config* cfg, vsa_clip** out);

/* Wait for the analyser's work and free it.  NULL is a no-op. */
void vsa_clip_destroy(vsa_clip* c);

/* Analyse the n_frames frames of one clip; returns when every record is out.
 * Frame i is the plane at frames + i * frame_stride_bytes with rows
 * pitch_bytes apart, in host memory (src = VSA_SRC_HOST: uploaded chunk by
 * chunk) or device memory (VSA_SRC_DEVICE_BORROW: read in place; the caller
 * keeps it valid until the call returns).  out_frames receives n_frames
 * records in frame order (pts = frame index); out_shots the first shots_cap
 * shot records, and *n_shots (nullable) the clip's shot count, which may
 * exceed shots_cap (n_frames + 1 always suffices).  Both arrays are the
 * caller's.  n_frames = 0 gives no records and no shots.  Errors: VSA_E_INVAL
 * (NULL, pitch below a row, stride below a frame, bad src), VSA_E_NOMEM,
 * VSA_E_DEVICE.  Calls on one analyser are serialised. */
vsa_status vsa_clip_run(vsa_clip* c, const void* frames, int64_t frame_stride_bytes, int64_t pitch_bytes,
                        int32_t n_frames, int32_t src, vsa_frame_result* out_frames,
                        vsa_shot_result* out_shots, int32_t shots_cap, int32_t* n_shots);

/* Instrumentation (not in the paper): the first n of [0] chunks processed,
 * [1] decision launches (one per chunk plus one per round), [2] host waits,
 * [3] sparse pair tasks computed, [4] of those, speculative field measures
 * (computed ahead of the pass; some may never be asked for), [5] sparse
 * measures the sequential pass requested (Sec. III.A's selective schedule:
 * field measures served from the speculative cache count as requested),
 * summed over the analyser's runs. */
vsa_status vsa_clip_counters(vsa_clip* c, uint64_t* out, int32_t n);

/* Test hook: the sparse measures the sequential pass requested in the last
 * run of an analyser created with debug_log, up to cap x 6 int32 (kind, ref,
 * oth, ref_field, oth_field, level; the caller's array), the same set the
 * oracle logs in the sparse schedule.  Returns the count, VSA_E_STATE without
 * debug_log, VSA_E_INVAL for bad arguments. */
int32_t vsa_clip_debug_log(vsa_clip* c, int32_t* keys, int32_t cap);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the pair measure of
 * vsa_debug_pair (motion field, exact moments, NCC, SWR, AMM, ACT; Sec. III.A)
 * on two w x h planes already in device memory, with nothing allocated.  Every
 * intermediate lives in one fixed device array of the library (about 4 MiB,
 * held on each GPU the library runs on until the process ends); the call only
 * enqueues kernels on hip_stream (nullable: the null stream) on the calling
 * thread's current device and returns without waiting.
 *   I, J          planes of uint8 (bit_depth 8) or uint16 samples <= 1023 (bit_depth
 *                 10, 2-byte aligned), rows pitch_bytes apart; read, not kept
 *   w, h          8..1024 each (larger: VSA_E_INVAL, the array's limit)
 *   mv            device, (w/8)*(h/8) x 2 int8 (dx, dy per block), or NULL
 *   ints          device, 9 int64: Sx, Sy, Sxx, Syy, Sxy, N, A, B, STATIC; or NULL
 *   dbl           device, 4 doubles: NCC, SWR, AMM, ACT; or NULL
 * The outputs are the caller's and are written when the stream reaches the
 * work.  All calls on one GPU share the array: calls that may overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Errors: VSA_E_INVAL (NULL plane, size, pitch, alignment, bit depth),
 * VSA_E_UNSUPPORTED (block or radius other than 8, or search other than 0:
 * the full search only), VSA_E_DEVICE. */
vsa_status vsa_pair_noalloc(const vsa_params* p, const void* I, const void* J, int32_t w, int32_t h,
                            int64_t pitch_bytes, int32_t bit_depth, int32_t force_zero_mv, int8_t* mv,
                            int64_t* ints, double* dbl, void* hip_stream);

/* Thread-local description of the last error; valid until the next call. */
const char* vsa_last_error(void);

/* ---- test hooks: run one kernel in isolation on host buffers ------------- */

/* Pyramid and fields of one frame (Sec. III.C): frame levels L..Ltop
 * (Ltop = min(L + 4, Lcap)) then
 * the upper and lower field at Lf, densely packed as uint16, in that order.
 * *n_out receives the sample count (call with out = NULL to size). */
vsa_status vsa_debug_levels(const vsa_params* p, const void* luma, int32_t width, int32_t height,
                            int64_t pitch_bytes, int32_t bit_depth, uint16_t* out, int64_t cap,
                            int64_t* n_out);

/* Pair measure (Sec. III.A) of two w x h planes (uint16 samples, densely packed):
 * mv (B x 2 int8), sad (B int32, nullable), ints (Sx, Sy, Sxx, Syy, Sxy, N, A,
 * B, STATIC), dbl (NCC, SWR, AMM, ACT).  bit_depth selects the 8-bit or
 * 10-bit kernel; force_zero_mv uses d = (0, 0) for every block.  The block
 * searches only (search 0 or 1; 2 is VSA_E_UNSUPPORTED: vsa_debug_flow_pair). */
vsa_status vsa_debug_pair(const vsa_params* p, const uint16_t* I, const uint16_t* J, int32_t w,
                          int32_t h, int32_t bit_depth, int32_t force_zero_mv, int8_t* mv,
                          int32_t* sad, int64_t* ints, double* dbl);

/* Dense inverse search flow pair measure (Sec. III.A: the paper's motion
 * field is dense inverse search optical flow, its reference [8]), with fixed
 * work so that it is exactly reproducible: the pair's planes and up to two
 * 2x2-box-downscaled copies, coarsest first; 8 x 8 patches every 4 samples
 * (plus one flush with the right and bottom edges); per patch eight
 * inverse-compositional steps u <- u - H^-1 sum g (J(x + u) - T(x)),
 * H = sum g g^T + 64 I, central-difference gradients, J sampled bilinearly
 * with clamped coordinates, components clamped to +-32; the flow at a pixel
 * is the mean of the covering patches' vectors weighted by
 * 1 / max(1, |J(x + u) - I(x)|).  Measures: NCC of I against J warped by the
 * flow over every pixel, SWR = 1 - NCC, AMM = mean flow length (pixels of
 * the plane), ACT = sqrt((AMM + a0) SWR); static if 256 AMM < a_static_fx.
 * IEEE double, sums in a fixed order: the results are bitwise those of the
 * sequential definition.
 *
 * vsa_flow_scratch_bytes: device bytes the measure of a w x h pair needs
 * (w, h >= 8, fewer than 2^31 samples), or VSA_E_INVAL.
 * vsa_flow_pair: I, J device planes of w x h samples (bits 8: bytes, 10:
 * uint16 words, 2-byte aligned) with a row pitch in bytes; scratch: device
 * memory of at least vsa_flow_scratch_bytes (the caller's, not kept);
 * flow: device w x h x 2 doubles (dx, dy interleaved, pixels of the plane) or
 * NULL; results: device 5 doubles (NCC, SWR, AMM, ACT, static 0/1).  Only
 * a0 and a_static_fx of p are read (NULL = defaults).  Enqueued on
 * hip_stream (NULL = the null stream); no allocation, no synchronisation.
 * vsa_debug_flow_pair: the same from host planes of uint16 samples (w x h,
 * dense), synchronous; flow (w x h x 2, nullable), dbl (NCC, SWR, AMM, ACT),
 * is_static (nullable) are host arrays. */
int64_t vsa_flow_scratch_bytes(int32_t w, int32_t h);
vsa_status vsa_flow_pair(const vsa_params* p, const void* I, const void* J, int32_t w, int32_t h,
                         int64_t pitch_bytes, int32_t bits, void* scratch, int64_t scratch_bytes,
                         double* flow, double* results, void* hip_stream);
vsa_status vsa_debug_flow_pair(const vsa_params* p, const uint16_t* I, const uint16_t* J, int32_t w,
                               int32_t h, int32_t bits, double* flow, double* dbl, int32_t* is_static);

/* How vsa_clip_run splits an n_frames clip at this chunk size (0 = 256):
 * chunk i covers frames starts[i] .. starts[i] + counts[i] - 1, for the first
 * min(count, cap) chunks (arrays of cap entries, the caller's; NULL with cap
 * 0 to count).  Host arithmetic only.  Returns the chunk count, or
 * VSA_E_INVAL. */
int32_t vsa_debug_clip_chunks(int32_t chunk, int32_t n_frames, int32_t* starts, int32_t* counts, int32_t cap);

/* The finishing arithmetic of Sec. III.A on n integer tuples
 * (Sx, Sy, Sxx, Syy, Sxy, N, A, B) -> n x (NCC, SWR, AMM, ACT), computed by the
 * device (ints: n x 8 int64; out: n x 4 double; both the caller's). */
vsa_status vsa_debug_finish(const int64_t* ints, int64_t n, double a0, double* out);

/* Decision logic alone (Sec. III.B-D), driven by injected measure sequences
 * instead of frames (act, swr, stat: T; v: T x 3 (v0, v1, v2); F, S, P:
 * T x (k_max + 2), column K the forward ACT, its SWR and the backward ACT at
 * distance K).  Runs the device state machine one
 * simulated frame arrival at a time.  recs: T records; shots: up to shots_cap;
 * keys (nullable): up to keys_cap x 6 int32 (kind, ref, oth, ref_field,
 * oth_field, level) of the sparse measures requested. */
vsa_status vsa_debug_decide(const vsa_params* p, int32_t k_max, int32_t dense, int32_t T,
                            const double* act, const double* swr, const uint8_t* stat,
                            const double* v, const double* F, const double* S, const double* P,
                            vsa_frame_result* recs, vsa_shot_result* shots, int32_t shots_cap,
                            int32_t* n_shots, int32_t* keys, int32_t keys_cap, int32_t* n_keys);

/* Sparse measures computed for stream sid (engines created with debug_log):
 * up to cap x 6 int32 as in vsa_debug_decide; returns the count or < 0. */
int32_t vsa_debug_measure_log(vsa_engine* e, int32_t sid, int32_t* keys, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
