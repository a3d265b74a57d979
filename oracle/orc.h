/*
 * orc.h -- C ABI of the CPU oracle for the per-frame measure engine.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded scalar
 * implementation of what the engine computes, written from the paper's
 * definitions (Fassold, "Faster than real-time detection of shot boundaries,
 * sampling structure and dynamic keyframes in video", Sec. III).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code with the GPU library.
 *
 * Conventions: every call returns 0 on success or a negative code
 * (-1 invalid argument, -2 out of memory, -3 output capacity too small).
 * The caller owns every buffer.  Planes are row-major; `pitch` arguments
 * are in bytes.  Pixel values are 8-bit (uint8 storage) or 10-bit
 * (uint16 storage, values <= 1023).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm constants; the paper prints none, so every value is an input. */
typedef struct {
    int32_t block;        /* block edge in pixels (8)                          */
    int32_t radius;       /* full-search radius R in working pixels (8)        */
    int32_t wmax;         /* working level: first level with width <= wmax     */
    int32_t lf_offset;    /* field level = max(0, L - lf_offset)               */
    int32_t k_max;        /* longest dissolve searched by the deep check       */
    int32_t a_static_fx;  /* STATIC if A < a_static_fx * B (A in 1/256 px)     */
    int32_t w_hist;       /* fast-check history length                         */
    int32_t n_ss;         /* frames analysed per shot for sampling structure   */
    double a0;            /* ACT = sqrt((AMM + a0) * SWR)                       */
    double rho_f, theta_f;/* fast check: a > rho_f * mean(hist) + theta_f      */
    double theta_f0;      /* fast check with an empty history: a > theta_f0    */
    double rho_d, theta_d;/* deep check: F > rho_d * P + theta_d               */
    double gamma;         /* plateau rule for the dissolve length              */
    double tau_c;         /* comb tests: v0 > tau_c * min(v1, v2) (interlace) and
                             v0 > tau_c * max(v1, v2) (pulldown cadence)      */
    double eps;           /* class fraction margin                             */
    double tau_p;         /* pulldown: combed positions' mean v0 ratio          */
    double theta_kf;      /* keyframe threshold on accumulated ACT             */
    int32_t search;       /* motion field: 0 full search over [-R, R]^2 (every pair);
                             1 coarse-to-fine for frame pairs: full search on the 2x2-box
                             image one level coarser, then +-refine around twice that
                             vector (field pairs: full search);
                             2 dense inverse search flow for every pair (orc_flow_pair) */
    int32_t refine;       /* refinement radius r of the coarse-to-fine search   */
} orc_params;

/* Per-frame record. */
typedef struct {
    int64_t frame;
    int32_t flags;        /* ORC_F_* bits                                      */
    int32_t shot_id;      /* -1 for frames inside a transition                 */
    int32_t boundary;     /* 0 none, 1 hardcut, 2 dissolve (set on first frame of the new shot) */
    int32_t boundary_k;   /* K* of that boundary                               */
    double ncc, swr, amm, act;      /* of the pair (frame -> frame+1)          */
    int64_t mom[5];                 /* Sx, Sy, Sxx, Syy, Sxy                   */
    int64_t n_pix, amm_num;         /* N = 64 B and A                          */
    int32_t n_blocks;
    uint32_t field_mask;            /* bit i set if v_i was computed           */
    double v[3];                    /* v0, v1, v2 (NaN if not computed)        */
    double h_mean, h_std, h_mad;    /* intensity measures of the frame (working level) */
} orc_frame_rec;

enum {
    ORC_F_HAS_PAIR = 1, ORC_F_STATIC = 2, ORC_F_FAST_FIRED = 4,
    ORC_F_IN_TRANSITION = 8, ORC_F_KEYFRAME = 16, ORC_F_SHOT_START = 32,
    ORC_F_ANALYZED = 64
};

typedef struct {
    int32_t shot_id, pad0;
    int64_t first, last;
    int32_t in_boundary, in_k;
    int32_t sampling;       /* 0 undetermined, 1 progressive, 2 TFF, 3 BFF, 4 pulldown 3:2 */
    int32_t pulldown_phase; /* -1 unless pulldown                               */
    int32_t n_analyzed, final_;
} orc_shot_rec;

/* Sec. III.A, the unary intensity measure H(t): the histogram of a plane
 * (w x h samples, row-major, values < 2^bits) and the mean, the standard
 * deviation and the mean absolute deviation (about the mean) taken from it.
 * hist: 2^bits counts; ints: N, S1 = sum v h[v], S2 = sum v^2 h[v],
 * M = sum h[v] |N v - S1|; out3: mean, std, mad.  Any output may be NULL. */
int32_t orc_intensity(const uint16_t* px, int32_t w, int32_t h, int32_t bits, int64_t* hist, int64_t* ints,
                      double* out3);

/* Key of one computed pair measure: ref -> oth, each a frame (field 0),
 * its upper field (1) or its lower field (2), at pyramid level `level`.
 * kind: 0 consecutive, 1 field pair, 2 deep check forward, 3 deep check backward. */
typedef struct { int32_t kind, ref, oth, ref_field, oth_field, level; } orc_measure_key;

/* Geometry of a W x H clip: out[0]=L, out[1]=Lcap, out[2]=Lf, out[3]=number of
 * frame levels (Lcap+1), then for l=0..Lcap: (w_l, h_l) at out[4+2l], and the
 * field level size (wf, hf) after that.  cap = length of out. */
int32_t orc_geometry(int32_t W, int32_t H, const orc_params* p, int32_t* out, int32_t cap);

/* One 2x2 rounding downscale step of a w x h plane (uint16 samples). */
int32_t orc_downscale(const uint16_t* src, int32_t w, int32_t h, uint16_t* dst);

/* All levels of one frame, as uint16: frame levels L..Lcap, then U_Lf, D_Lf
 * and the lower field resampled to the upper field's rows (the plane field
 * pairs read), concatenated, each densely packed (pitch = width). Returns the
 * number of samples written in *n_out. */
int32_t orc_levels(const void* Y, int32_t W, int32_t H, int64_t pitch_bytes, int32_t bits,
                   const orc_params* p, uint16_t* out, int64_t cap, int64_t* n_out);

/* Pair measure M(I -> J) at one level (I, J: w x h uint16, densely packed),
 * with the motion field of p->search (the plane pair is taken as a frame pair).
 * mv: B x 2 int8 (dx, dy); sad: B int32 (nullable);
 * ints: Sx, Sy, Sxx, Syy, Sxy, N, A, B, STATIC;  dbl: NCC, SWR, AMM, ACT.
 * force_zero_mv = 1 skips the search and uses d = (0, 0) for every block. */
int32_t orc_pair(const uint16_t* I, const uint16_t* J, int32_t w, int32_t h,
                 const orc_params* p, int32_t force_zero_mv,
                 int8_t* mv, int32_t* sad, int64_t* ints, double* dbl);

/* NCC, SWR, AMM, ACT from the exact integers (Sx, Sy, Sxx, Syy, Sxy, N, A, B). */
/* Pair measure with the dense inverse search flow (search = 2): flow (w x h
 * x 2 doubles: dx, dy per pixel; nullable), dbl: NCC, SWR, AMM, ACT,
 * *is_static (nullable).  Planes at least 8 x 8. */
int32_t orc_flow_pair(const uint16_t* I, const uint16_t* J, int32_t w, int32_t h, const orc_params* p,
                      double* flow, double* dbl, int32_t* is_static);

int32_t orc_finish(const int64_t* ints8, double a0, double* out4);

/* The offline sequential pass over a whole clip.  frames: T planes of
 * W x H samples at the given pitch, frame_stride bytes apart.  dense = 1
 * computes every field and deep-check measure at every iteration (labels
 * are unchanged).  mv_out (nullable) receives (T-1) x B x 2 int8 of the
 * consecutive pairs at the working level. */
int32_t orc_run_clip(const void* frames, int32_t T, int32_t W, int32_t H, int64_t pitch_bytes,
                     int64_t frame_stride_bytes, int32_t bits, int32_t dense, const orc_params* p,
                     orc_frame_rec* recs, orc_shot_rec* shots, int32_t shots_cap, int32_t* n_shots,
                     orc_measure_key* keys, int32_t keys_cap, int32_t* n_keys, int8_t* mv_out);

/* The same pass driven by injected measure sequences instead of frames.
 * act, swr: T (entry t = pair t -> t+1, T-1 used); stat: T; v: T x 3;
 * F, S, P: T x (k_max + 2), entry [t][K] for K = 1..k_max+1 ([t][1] of F and S
 * must equal act[t] and swr[t]).  P[t][K] is used only when
 * min(K, t - shot_start) > 0, otherwise 0.0 is taken. */
int32_t orc_decide_injected(int32_t T, const double* act, const double* swr, const uint8_t* stat,
                            const double* v, const double* F, const double* S, const double* P,
                            int32_t dense, const orc_params* p, orc_frame_rec* recs,
                            orc_shot_rec* shots, int32_t shots_cap, int32_t* n_shots,
                            orc_measure_key* keys, int32_t keys_cap, int32_t* n_keys);

#ifdef __cplusplus
}
#endif
#endif
