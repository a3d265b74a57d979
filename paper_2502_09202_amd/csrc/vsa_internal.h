// vsa_internal.h -- device-side data layout shared by the HIP kernels and the
// host runtime of libvsa (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "../../include/vsa.h"

namespace vsa {

constexpr int kBlock = 8;           // block edge (pixels)
constexpr int kRadius = 8;          // full-search radius (working pixels)
constexpr int kCand = 2 * kRadius + 1;
constexpr int kMaxLevels = 5;       // frame levels stored per ring slot: L .. L+4
constexpr int kMaxKmax = 15;
constexpr int kMaxHist = 16;
constexpr int kMaxStreams = 1024;
constexpr int kDecideWaves = 1;         // decision kernel: one wavefront per stream and per workgroup
                                        // (small workgroups are placed at once beside the persistent
                                        // motion-search grids; 8-wave ones waited for room)

// Field selector of a plane inside a ring slot.
enum : int32_t { PL_FRAME = 0, PL_UPPER = 1, PL_LOWER = 2 };

// Measure kinds (also the "kind" of a logged key).
enum : int32_t { MK_CONSEC = 0, MK_FIELD = 1, MK_DEEP_F = 2, MK_DEEP_P = 3 };

// Geometry and device addresses of one open stream.
struct StreamDesc {
    int32_t active;
    int32_t W, H, bits;
    int32_t L, Lcap, Lf, ltop;        // frame levels L..ltop are stored
    int32_t nlev;                     // ltop - L + 1
    int32_t k_max;
    int32_t rs;                       // ring slots (frames held)
    int32_t wl[kMaxLevels], hl[kMaxLevels], pl[kMaxLevels];   // size and pitch (samples) per stored level
    int64_t off[kMaxLevels];          // byte offset of each stored level in a slot
    int32_t wf, hf, pf;               // field level size and pitch
    int64_t offU, offD;               // byte offsets of the fields in a slot
    int64_t offH;                     // byte offset of the frame's intensity histogram (2^bits uint32)
    int64_t slot_bytes;
    uint8_t* ring;                    // rs slots
    struct FrameInfo* info;           // rs entries
    int8_t* mv;                       // rs x (B_L x 2)
    uint16_t* tileh;                  // per pyramid tile: its working-level histogram (2^bits counts)
    int32_t B_L;                      // blocks at the working level
    int32_t epoch;                    // bumped each time the slot is (re)opened
    int32_t search;                   // 0 full search, 1 coarse-to-fine (frame pairs), 2 dense flow
};

// Per-frame record under construction (one per ring slot).
struct FrameInfo {
    int64_t frame, pts;
    int32_t flags, shot_id, boundary, boundary_k;
    double ncc, swr, amm, act;
    int64_t mom[5];
    int64_t n_pix, amm_num;
    int32_t n_blocks;
    uint32_t field_mask;
    double v[3];
    double h_mean, h_std, h_mad;      // intensity measures of the frame (working level)
};

// One pair measure to compute: ref -> oth planes of stream `sid`.
struct PairTask {
    int32_t sid;
    int32_t kind;                     // MK_*
    int32_t ref, oth;                 // frame indices
    int32_t ref_field, oth_field;     // PL_*
    int32_t level;                    // absolute pyramid level
    int32_t result;                   // index into the stream's sparse result slots (-1: consecutive)
    int32_t tiles;                    // ME tiles of the pair
    int32_t tile_prefix;              // first tile of the pair within its list
    int32_t flags;                    // TF_*
    int32_t epoch;                    // StreamDesc::epoch when planned; stale tasks are skipped
};

enum : int32_t {
    TF_MV_RING = 1,    // store the motion field in the stream's MV ring (consecutive pairs)
    TF_DEBUG = 2,      // store motion field, SADs and integers in the debug buffers
    TF_ZERO_MV = 4,    // use d = (0, 0) for every block (no search)
    TF_HIER = 8,       // coarse-to-fine motion field, 16 x 16-block tiles (frame pairs of a
                       // stream whose parameters ask for it)
    TF_FLOW = 16       // dense flow pair measure, one tile per row of the plane (every pair
                       // of a stream whose parameters ask for it)
};

// Result of a sparse pair measure.
struct PairResult {
    double act, swr;
};

// Sparse result slots of a stream: fields (3), deep forward F_K and deep
// backward P_K for K = 1..kMaxKmax+1.
constexpr int kResFields = 0;
constexpr int kResF = 3;
constexpr int kResP = kResF + kMaxKmax + 2;
constexpr int kResSlots = kResP + kMaxKmax + 2;
// Speculative field measures (offline clip form only): when an iteration
// asks for the fields of its frame, those of up to kMaxSpec later frames the
// analysis may still want are computed with them and cached per ring slot.
// Their tasks carry result = kResSpec + component.
constexpr int kMaxSpec = 10;
constexpr int kResSpec = kResSlots;
static_assert(3 + 3 * kMaxSpec <= 3 + 2 * (kMaxKmax + 1), "speculative tasks exceed the per-stream task limit");

// Sampling-structure analysis of the open shot.
struct Analysis {
    int32_t open, n, nci, s, result, phase;
    int32_t np[5], pad;         // analysed frames per position of the 5-frame unit
    double s0[5];               // sum of v0 per position
    double sum1, sum2;
};

// Decision state of one stream.
struct DecideState {
    int32_t t;                  // next iteration of the sequential pass
    int32_t n;                  // newest frame index ingested (-1: none)
    int32_t T_end;              // total frames once the stream has ended, else -1
    int32_t emitted;            // frames [0, emitted) have been written out
    int32_t shot_start, shot_id;
    int32_t hist_len, hist_pad;
    double hist[kMaxHist];      // the last hist_len values end at index kMaxHist-1 (oldest first)
    double acc;                 // keyframe accumulator
    Analysis ss;
    int32_t cur_in_boundary, cur_in_k;   // how the current shot began
    // iteration planned in the previous step (its sparse measures are computed
    // by this step's motion-search launch)
    int32_t plan, plan_want, plan_fire, plan_deep, plan_nf, plan_kn;
    int32_t plan_spec;                   // speculative field frames planned with it:
    uint32_t spec_mask;                  // bit k = frame t + 1 + k
    int32_t spec_next, spec_pad;         // frames below spec_next were considered for speculation
    int32_t done;               // end of stream fully processed
    int32_t n_closed;           // shots closed by the last advance
    int32_t sp_base, sp_count;  // where the planned tasks sit in that step's sparse list
    int64_t log_count;          // sparse measures requested by the pass (logged when a log is kept)
    int64_t spec_count;         // speculative field tasks planned (offline clip form)
};

// Shots closed by one advance of a stream: at most 3 (a planned boundary, one
// immediate boundary at the clip end, the last shot).
constexpr int kMaxClosed = 4;

// Engine-wide constants for the decision kernel.
struct DecideParams {
    int32_t w_hist, n_ss, dense, a_static_fx;
    double a0, rho_f, theta_f, theta_f0, rho_d, theta_d, gamma, tau_c, eps, tau_p, theta_kf;
    // field cache of the speculative field measures: per ring slot v0, v1, v2
    // and the frame they belong to (NaN: none); null disables speculation
    double* spec;
};

// Per-step view of one stream (host -> device each step).
struct StepStream {
    int32_t sid;
    int32_t has_frame;          // a frame was pushed for this step
    int32_t frame;              // its index
    int32_t ended_T;            // total frame count if the stream has ended, else -1
    int64_t pts;
    const void* src;            // plane to ingest
    int64_t src_pitch;          // bytes
    int32_t k1_tiles;           // pyramid tiles of this stream
    int32_t k1_prefix;          // first pyramid tile
    int32_t consec_tiles;       // ME tiles of its consecutive pair (0 if none)
    int32_t consec_prefix;      // first tile (and partial) of that pair
};

// Output ring entries (device -> host).
struct OutFrame {
    int32_t sid, pad;
    vsa_frame_result r;
};
struct OutShot {
    int32_t sid, pad;
    vsa_shot_result r;
};

// Counters and cursors in device memory.
// Each counter sits on its own 128-byte line so that concurrent atomics on
// different counters do not serialise on one line.
struct alignas(128) DeviceCounter {
    unsigned long long v;
    unsigned long long pad[15];
};

struct DeviceCursors {
    DeviceCounter frames_written;    // monotonically increasing write cursor (OutFrame ring)
    DeviceCounter shots_written;
    // sparse tasks planned by the decision kernel of steps of parity p, packed
    // as (tasks << 32 | tiles); the next step's motion search reads it (and
    // clears the other entry before that step's decisions add to it)
    DeviceCounter sparse_tt[2];
    DeviceCounter sparse_run;        // total sparse tasks planned
    DeviceCounter sparse_blocks;     // total 8x8 blocks of those tasks
    DeviceCounter blocks_done;       // workgroups of the running decision kernel that finished
};

// Output cursors as of the end of one step, written by the last workgroup of
// the step's decision kernel into mapped host memory (what vsa_collect reads).
// Optional event pair of a kernel launch (hipExtLaunchKernel): start is
// stamped when the kernel begins, stop when it ends, from the dispatch itself
// rather than from separate marker packets.  Either may be null; with both
// null the launch takes the plain (cheaper on the host) path.
struct LaunchTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    bool any() const { return start != nullptr || stop != nullptr; }
};

struct PubSnap {
    uint64_t frames_written, shots_written, sparse_run, sparse_blocks;
};

__host__ __device__ inline int tt_tasks(unsigned long long v) { return (int)(v >> 32); }
__host__ __device__ inline int tt_tiles(unsigned long long v) { return (int)(v & 0xffffffffu); }

// ME tiling: a tile is TBX x TBY blocks, one 256-thread workgroup.
constexpr int kTBX = 8;
constexpr int kTBY = 8;
constexpr int kMEThreads = 256;

inline __host__ __device__ int div_up(int a, int b) { return (a + b - 1) / b; }
inline __host__ __device__ int me_tiles(int w, int h) {
    return div_up(w / kBlock, kTBX) * div_up(h / kBlock, kTBY);
}
// Coarse-to-fine tiles are 16 x 16 blocks (their coarse level, 8 x 8 blocks,
// has the full search's tile shape).
constexpr int kHTB = 16;
inline __host__ __device__ int me_tiles_hier(int w, int h) {
    return div_up(w / kBlock, kHTB) * div_up(h / kBlock, kHTB);
}
// Tiles of a frame pair and of a field pair.  The dense flow's tiles are
// the plane's rows; the coarse-to-fine search leaves field pairs to the full
// search.
inline __host__ __device__ int frame_pair_tiles(int search, int w, int h) {
    return search == 2 ? h : (search ? me_tiles_hier(w, h) : me_tiles(w, h));
}
inline __host__ __device__ int field_pair_tiles(int search, int w, int h) {
    return search == 2 ? h : me_tiles(w, h);
}

// Everything a motion-search tile needs from its pair, resolved once per pair
// by the pair's producer (the pyramid kernel for the consecutive pair of a
// step, the decision kernel for the sparse pairs it plans), so that a tile is
// found with two loads: the tile's job index from a per-tile map, then the job.
struct TileJob {
    const uint8_t* I;                 // reference plane (its blocks tile the search)
    const uint8_t* J;                 // searched plane
    int8_t* mv;                       // motion-field destination, or null
    int32_t w, h, pitch;              // plane size and row pitch (samples), same for I and J
    int32_t cos_I, cos_J;             // 0, or Lf + 1: the lower field read on the upper field's rows
    int32_t tiles_x;                  // tiles per row of the plane
    int32_t tile_prefix;              // first tile of the pair within its list
    int32_t flags;                    // TF_*
    int32_t sid, epoch;               // stream and its epoch when planned
    int32_t bits;                     // 8 or 10
    // coarse-to-fine frame pairs: the pair's planes one level coarser when
    // the ring holds that level (the stored pyramid level is exactly the
    // 2 x 2 box image of the pair's level), else null
    const uint8_t* cI;
    const uint8_t* cJ;
    int32_t cpitch;                   // its row pitch (samples)
};

// Job of pair t of stream sd (mv: the motion-field destination).
inline __host__ __device__ TileJob make_tile_job(const StreamDesc& sd, const PairTask& t, int8_t* mv) {
    TileJob j;
    const int64_t sref = (int64_t)(t.ref % sd.rs) * sd.slot_bytes;
    const int64_t soth = (int64_t)(t.oth % sd.rs) * sd.slot_bytes;
    if (t.ref_field != PL_FRAME) {
        const int64_t oref = t.ref_field == PL_UPPER ? sd.offU : sd.offD;
        const int64_t ooth = t.oth_field == PL_UPPER ? sd.offU : sd.offD;
        j.I = sd.ring + sref + oref;
        j.J = sd.ring + soth + ooth;
        j.w = sd.wf; j.h = sd.hf; j.pitch = sd.pf;
        j.cos_I = t.ref_field == PL_LOWER ? sd.Lf + 1 : 0;
        j.cos_J = t.oth_field == PL_LOWER ? sd.Lf + 1 : 0;
    } else {
        const int d = t.level - sd.L;
        j.I = sd.ring + sref + sd.off[d];
        j.J = sd.ring + soth + sd.off[d];
        j.w = sd.wl[d]; j.h = sd.hl[d]; j.pitch = sd.pl[d];
        j.cos_I = j.cos_J = 0;
    }
    const bool hier = sd.search == 1 && t.ref_field == PL_FRAME;
    const bool flow = sd.search == 2;
    j.cI = j.cJ = nullptr;
    j.cpitch = 0;
    if (hier && t.level - sd.L + 1 < sd.nlev) {
        const int dc = t.level - sd.L + 1;
        j.cI = sd.ring + sref + sd.off[dc];
        j.cJ = sd.ring + soth + sd.off[dc];
        j.cpitch = sd.pl[dc];
    }
    j.mv = flow ? nullptr : mv;
    j.tiles_x = div_up(j.w / kBlock, hier ? kHTB : kTBX);
    j.tile_prefix = t.tile_prefix;
    j.flags = (flow ? (t.flags & ~TF_MV_RING) : t.flags) | (hier ? TF_HIER : 0) | (flow ? TF_FLOW : 0);
    j.sid = t.sid;
    j.epoch = t.epoch;
    j.bits = sd.bits;
    return j;
}

// Per-tile partial sums of a pair (exact integers).
struct TilePartial {
    int64_t sx, sy, sxx, syy, sxy, a;
};

// Pyramid tile: TW x TH pixels of the working level, 256 threads.
constexpr int kPyrTW = 64;
constexpr int kPyrTH = 16;

}  // namespace vsa
