// vsa_runtime.cpp -- host runtime and C ABI of libvsa (see include/vsa.h).
//
// One engine = one HIP stream of work on one device.  Every open stream owns
// one device allocation: a ring of 2 k_max + 7 frame slots (working level,
// the coarser levels used by the deep check and the two fields), the
// per-frame records under construction, the motion fields of the
// consecutive pairs, and two staging planes for copied input.  The engine
// owns the tables shared by all streams (stream descriptors, decision state,
// sparse results, the device-built sparse task list, tile partials and the
// output rings).
//
// A time step (vsa_step) enqueues, in order on the engine stream:
//   H2D   the step descriptor (which streams ingest which plane, the
//         consecutive-pair tasks) and any host-sourced planes;
//   K1    pyramid + fields of every ingested frame (one launch);
//   K2    motion search + moments over the consecutive pairs of this step
//         and the sparse pairs planned by the previous step (one persistent
//         launch per sample width);
//   K3    finish of every pair (NCC, SWR, AMM, ACT);
//   K6    decisions, sparse-task compaction for the next step, records.
// K1 and the uploads run on a second HIP stream ("ingest"); the rest on the
// main stream.  Step s's pyramid may run while steps s-3..s-1 are still in
// their motion search and decisions (the ring holds three extra slots and the
// step descriptor four copies for that), never further ahead.  The kernels
// stress different units (HBM vs VALU/latency), so they overlap well, and the
// main stream's wait for a pyramid is usually already satisfied.
// Nothing is copied back until vsa_sync, which drains the device output rings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "vsa_internal.h"

namespace vsa {
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s);
hipError_t launch_pyramid(int bits, int L, const StreamDesc*, const StepStream*, const int32_t*, int32_t, int32_t,
                          TileJob*, int32_t*, hipStream_t, LaunchTiming = {});
int pyramid_tiles(const StreamDesc& sd);
hipError_t launch_intensity(const StreamDesc*, const StepStream*, const int32_t*, int32_t, hipStream_t);
int me_max_wgs_per_cu(int bits);
hipError_t launch_me(int bits, const StreamDesc*, const TileJob*, int32_t, const int32_t*, int32_t,
                     const DeviceCursors*, int32_t, bool, TilePartial*, int8_t*, int32_t*, int grid, hipStream_t,
                     LaunchTiming = {});
int me_hier_max_wgs_per_cu(int bits);
int64_t flow_scratch_bytes(int w, int h);
hipError_t launch_flow_pair(const uint8_t* I, const uint8_t* J, int w, int h, int64_t pitch, int bits, double a0,
                            int a_static_fx, uint8_t* scratch, double* flow_out, double* res_out, hipStream_t s);
int64_t flow_pair_bytes(int w, int h);
hipError_t launch_flow_list(const StreamDesc*, const TileJob*, int32_t, const int32_t*, int32_t, const DeviceCursors*,
                            int32_t, bool, uint8_t*, int64_t, TilePartial*, int64_t tiles_bound, int cus, hipStream_t);
hipError_t launch_me_hier(int bits, const StreamDesc*, const TileJob*, int32_t, const int32_t*, int32_t,
                          const DeviceCursors*, int32_t, TilePartial*, int8_t*, int32_t*, int grid, hipStream_t,
                          LaunchTiming = {});
hipError_t launch_finish(const StreamDesc*, const PairTask*, int32_t, int32_t, const PairTask*,
                         DeviceCursors*, const TilePartial*, PairResult*, const DecideParams&, int64_t*,
                         double*, int grid, int32_t par_prev, hipStream_t);
hipError_t launch_finish_debug(const int64_t*, int64_t, double, double*, hipStream_t);
hipError_t launch_finish_decide(const StreamDesc*, DecideState*, const StepStream*, int32_t, const DecideParams&,
                                const TilePartial*, const TilePartial*, const PairTask*, PairTask*, DeviceCursors*,
                                OutFrame*,
                                uint64_t, OutShot*, uint64_t, int32_t*, int64_t, vsa_shot_result*, int32_t,
                                PubSnap*, TileJob*, int32_t*, hipStream_t, LaunchTiming = {});
hipError_t launch_decide_replay(const StreamDesc&, DecideState*, PairResult*, const DecideParams&, int32_t,
                                const double*, const double*, const uint8_t*, const double*, const double*,
                                const double*, const double*, vsa_frame_result*, vsa_shot_result*, int32_t,
                                int32_t*, int32_t*, int32_t, int32_t*, hipStream_t);
}  // namespace vsa

using namespace vsa;

namespace {

thread_local std::string g_err;

vsa_status fail(vsa_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

vsa_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return VSA_E_DEVICE;
}

}  // namespace

namespace vsa {
// error reporting for the library's other translation units
vsa_status report_error(vsa_status code, const char* msg) { return fail(code, msg); }
vsa_status report_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace vsa

namespace {

#define HIPCK(x, what)                                  \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr int kMaxTasksPerStream = 3 + 2 * (kMaxKmax + 1);
constexpr uint64_t kFramesCap = 1u << 16;
constexpr uint64_t kShotsCap = 1u << 16;
constexpr int kProfRing = 64;
// The ingest stream may run up to kAhead steps ahead of the main stream.
constexpr int kAhead = 3;
constexpr int kProfKinds = 6;
constexpr int kDescRing = 8;
// Cursor snapshots, one per step (a ring): the host may run at most kDescRing
// steps ahead of the device, so a snapshot is never rewritten while it is read.
constexpr int kSnap = 64;
// Motion-search launch candidates: workgroups per CU of the persistent grid
// of the consecutive pairs and of the sparse pairs.
struct TuneCand { int consec, sparse; };
constexpr int kTuneN = 4;
constexpr TuneCand kTuneCands[kTuneN] = {{2, 2}, {3, 3}, {2, 3}, {3, 2}};
constexpr int kTuneSamples = 3;
constexpr int kTuneWindow = 8;     // steps per timing window
// Windows start only after this many steps of an engine: the first steps
// are not representative (every stream opens a shot at once and asks for the
// fields of its first analysed frames; buffers grow).
constexpr int kTuneStart = 64;
constexpr int kTuneRing = 16;
constexpr int64_t kLogCapPerStream = 1 << 16;

int ceil_log2(int k) {
    int c = 0;
    while ((1 << c) < k) ++c;
    return c;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Geometry of a W x H stream (same definitions as the decision kernel uses).
struct Geo {
    int L = -1, Lcap = -1, Lf = 0, ltop = 0, nlev = 0;
    int wl[kMaxLevels] = {0}, hl[kMaxLevels] = {0};
    int wf = 0, hf = 0;
};

vsa_status make_geo(int W, int H, const vsa_params& p, int kmax, Geo& g) {
    if (W <= 0 || H <= 0) return fail(VSA_E_INVAL, "frame size must be positive");
    std::vector<int> ws, hs;
    for (int w = W, h = H; w > 0 && h > 0; w /= 2, h /= 2) { ws.push_back(w); hs.push_back(h); }
    g.L = -1;
    for (size_t l = 0; l < ws.size(); ++l)
        if (ws[l] <= p.wmax) { g.L = (int)l; break; }
    if (g.L < 0 || ws[g.L] / 8 < 2 || hs[g.L] / 8 < 2)
        return fail(VSA_E_INVAL, "working level smaller than a 2x2 grid of 8x8 blocks");
    if (g.L > 4) return fail(VSA_E_UNSUPPORTED, "frames wider than 16 x wmax are not supported");
    g.Lcap = g.L;
    for (size_t l = g.L + 1; l < ws.size(); ++l) {
        if (ws[l] / 8 >= 2 && hs[l] / 8 >= 2) g.Lcap = (int)l; else break;
    }
    g.Lf = std::max(0, g.L - 1);
    g.wf = W >> g.Lf;
    g.hf = (H / 2) >> g.Lf;
    if (g.wf < 8 || g.hf < 8) return fail(VSA_E_INVAL, "field level smaller than one block");
    g.ltop = std::min(g.L + ceil_log2(kmax + 1), g.Lcap);
    g.nlev = g.ltop - g.L + 1;
    if (g.nlev > kMaxLevels) return fail(VSA_E_UNSUPPORTED, "k_max too large");
    for (int d = 0; d < g.nlev; ++d) { g.wl[d] = ws[g.L + d]; g.hl[d] = hs[g.L + d]; }
    return VSA_OK;
}

vsa_status check_params(const vsa_params& p) {
    if (p.block != 8 || p.radius != 8) return fail(VSA_E_UNSUPPORTED, "block must be 8 and radius 8");
    if (p.lf_offset != 1) return fail(VSA_E_UNSUPPORTED, "lf_offset must be 1");
    if (p.wmax < 16) return fail(VSA_E_INVAL, "wmax must be >= 16");
    if (p.k_max < 1 || p.k_max > kMaxKmax) return fail(VSA_E_INVAL, "k_max must be in 1..15");
    if (p.w_hist < 1 || p.w_hist > kMaxHist) return fail(VSA_E_INVAL, "w_hist must be in 1..16");
    if (p.n_ss < 1) return fail(VSA_E_INVAL, "n_ss must be >= 1");
    if (!(p.tau_p >= 1.0)) return fail(VSA_E_INVAL, "tau_p must be >= 1");
    if (p.search < 0 || p.search > 2) return fail(VSA_E_INVAL, "search must be 0, 1 or 2");
    if (p.search == 1 && p.refine != 1) return fail(VSA_E_UNSUPPORTED, "the coarse-to-fine search refines by 1");
    return VSA_OK;
}

DecideParams decide_params(const vsa_params& p, int dense) {
    DecideParams d;
    d.w_hist = p.w_hist; d.n_ss = p.n_ss; d.dense = dense; d.a_static_fx = p.a_static_fx;
    d.a0 = p.a0; d.rho_f = p.rho_f; d.theta_f = p.theta_f; d.theta_f0 = p.theta_f0; d.rho_d = p.rho_d; d.theta_d = p.theta_d;
    d.gamma = p.gamma; d.tau_c = p.tau_c; d.eps = p.eps; d.tau_p = p.tau_p; d.theta_kf = p.theta_kf;
    d.spec = nullptr;
    return d;
}

// Lay out one ring slot and fill the device descriptor (addresses excluded).
void layout(const Geo& g, int W, int H, int bits, int kmax, StreamDesc& sd) {
    std::memset(&sd, 0, sizeof sd);
    const int b = bits == 8 ? 1 : 2;
    sd.active = 1;
    sd.W = W; sd.H = H; sd.bits = bits;
    sd.L = g.L; sd.Lcap = g.Lcap; sd.Lf = g.Lf; sd.ltop = g.ltop; sd.nlev = g.nlev;
    sd.k_max = kmax;
    sd.rs = 2 * kmax + 4 + kAhead;   // deep-check look-back + look-ahead, + the pyramids running ahead
    int64_t off = 0;
    for (int d = 0; d < g.nlev; ++d) {
        sd.wl[d] = g.wl[d]; sd.hl[d] = g.hl[d];
        sd.pl[d] = (int)round_up(g.wl[d], 64);
        sd.off[d] = off;
        off = round_up(off + (int64_t)sd.pl[d] * g.hl[d] * b, 256);
    }
    sd.wf = g.wf; sd.hf = g.hf; sd.pf = (int)round_up(g.wf, 64);
    sd.offU = off;
    off = round_up(off + (int64_t)sd.pf * g.hf * b, 256);
    sd.offD = off;
    off = round_up(off + (int64_t)sd.pf * g.hf * b, 256);
    sd.offH = off;
    off = round_up(off + (int64_t)sizeof(uint32_t) * (1 << bits), 256);
    sd.slot_bytes = off;
    sd.B_L = (g.wl[0] / 8) * (g.hl[0] / 8);
}

// The moments and the intensity sums are exact 64-bit integers: refuse
// frames whose sums could overflow.
vsa_status check_exact_sums(const StreamDesc& sd) {
    // covariance terms need N (Sxx) products to stay below 2^63
    const int64_t maxv = sd.bits == 8 ? 255 : 1023;
    const int64_t nmax = 64LL * std::max<int64_t>((int64_t)(sd.wf / 8) * (sd.hf / 8), sd.B_L);
    if ((double)nmax * (double)nmax * (double)(maxv * maxv) >= 9.2e18)
        return fail(VSA_E_UNSUPPORTED, "frame too large for exact 64-bit moments");
    // and the intensity sums over the working level (N S2 < 2^63)
    const double npx = (double)sd.wl[0] * (double)sd.hl[0];
    if (npx * npx * (double)(maxv * maxv) >= 9.2e18)
        return fail(VSA_E_UNSUPPORTED, "frame too large for exact 64-bit intensity sums");
    return VSA_OK;
}

// Every sample of a 10-bit plane (uint16, rows pitch bytes apart) is <= 1023.
bool samples_10bit_ok(const uint8_t* plane, int64_t pitch, int W, int H) {
    uint16_t any = 0;
    for (int y = 0; y < H; ++y) {
        const uint16_t* r = reinterpret_cast<const uint16_t*>(plane + y * pitch);
        for (int x = 0; x < W; ++x) any |= r[x];
    }
    return (any & 0xFC00u) == 0;
}

int max_sparse_tiles(const StreamDesc& sd) {
    int n = 3 * field_pair_tiles(sd.search, sd.wf, sd.hf);
    for (int K = 1; K <= sd.k_max + 1; ++K) {
        const int l = std::min(sd.L + ceil_log2(K), sd.Lcap);
        const int d = l - sd.L;
        n += (K >= 2 ? 2 : 1) * frame_pair_tiles(sd.search, sd.wl[d], sd.hl[d]);
    }
    return n;
}

// Scratch bytes per tile of a stream's dense flow pairs (search 2): each of
// its pair planes (the stored frame levels and the field level) fits in its
// rows' share.  0 for the block searches.
int64_t flow_unit(const StreamDesc& sd) {
    if (sd.search != 2) return 0;
    int64_t u = 0;
    auto one = [&](int w, int h) { u = std::max(u, ((flow_pair_bytes(w, h) + h - 1) / h + 255) / 256 * 256); };
    for (int d = 0; d < sd.nlev; ++d) one(sd.wl[d], sd.hl[d]);
    one(sd.wf, sd.hf);
    return u;
}

// Device bytes a stream adds to the engine's per-tile buffers: its tile
// partials and, with the dense flow, its share of the flow scratch.
uint64_t stream_tile_bytes(const StreamDesc& sd) {
    const uint64_t tiles = (uint64_t)(frame_pair_tiles(sd.search, sd.wl[0], sd.hl[0]) + max_sparse_tiles(sd));
    return tiles * (sizeof(TilePartial) + (uint64_t)flow_unit(sd));
}

struct HostStream {
    bool open = false;
    vsa_stream_desc desc{};
    StreamDesc sd{};
    Geo geo;
    uint8_t* mem = nullptr;
    uint64_t mem_bytes = 0;    // size of mem
    uint64_t bytes = 0;        // budget charged (mem + tile partials)
    uint8_t* staging_dev[2] = {nullptr, nullptr};
    int64_t staging_pitch = 0;
    int next_frame = 0;        // frames pushed
    bool pending = false;      // a pushed frame waits for a step
    int pend_mode = 0;
    const void* pend_src = nullptr;
    int64_t pend_pitch = 0;
    int64_t pend_pts = 0;
    bool ended = false;
    int T_end = -1;
    int frames_out = 0;
    bool done = false;
    int consec_tiles = 0;
    int sparse_tiles_max = 0;
    int epoch = 0;
    std::deque<vsa_frame_result> fq;
    std::deque<vsa_shot_result> sq;
};

}  // namespace

struct vsa_engine {
    std::mutex mu;
    int device = 0;
    hipStream_t stream = nullptr;      // motion search, finish, decisions
    hipStream_t stream_b = nullptr;    // uploads and pyramid (one step ahead at most)
    hipStream_t stream_c = nullptr;    // motion search of the consecutive pairs
    hipEvent_t ev_c[kAhead + 1] = {};
    hipEvent_t ev_a[kAhead + 1] = {}, ev_b[kAhead + 1] = {};
    hipEvent_t ev_h[kAhead + 1] = {};   // the step's intensity measures are in the frame records
    int64_t step_no = 0;
    vsa_params params{};
    DecideParams dp{};
    int schedule = 0;
    int max_streams = 0;
    uint64_t budget = 0, used = 0;
    int debug_log = 0;
    std::vector<HostStream> streams;
    std::vector<int> slot_epoch;
    // engine-wide device tables
    StreamDesc* d_sds = nullptr;
    DecideState* d_states = nullptr;
    vsa_shot_result* d_closed = nullptr;
    PairResult* d_results = nullptr;
    PairTask* d_sparse = nullptr;
    DeviceCursors* d_cur = nullptr;
    OutFrame* d_out_frames = nullptr;
    OutShot* d_out_shots = nullptr;
    TilePartial* d_partials = nullptr;
    int64_t partials_cap = 0;
    // dense flow scratch (search 2): the consecutive pairs' and the sparse
    // pairs' lists, flow_unit bytes per tile (grown, never shrunk)
    uint8_t* d_flow_c = nullptr;
    uint8_t* d_flow_s = nullptr;
    int64_t flow_unit = 0, flow_tiles_c = 0, flow_tiles_s = 0;
    // motion-search jobs and tile maps: the consecutive pairs' per step slot
    // (written by the pyramid kernel), the sparse pairs' per step parity
    // (written by the decision kernel); maps hold partials_cap entries each
    TileJob* d_cjobs = nullptr;        // (kAhead + 1) x max_streams
    TileJob* d_sjobs = nullptr;        // 2 x max_streams x kMaxTasksPerStream
    int32_t* d_cmap = nullptr;         // (kAhead + 1) x partials_cap
    int32_t* d_smap = nullptr;         // 2 x partials_cap
    int32_t* d_log = nullptr;
    // step descriptors: device buffer + pinned host ring
    uint8_t* d_desc = nullptr;     // two step descriptors (alternating steps)
    uint8_t* h_desc[kDescRing] = {nullptr};       // pinned, mapped
    void* h_desc_dev[kDescRing] = {nullptr};      // device addresses of the same
    std::vector<uint8_t> desc_build;              // descriptors are built here (cached memory)
    hipEvent_t desc_ev[kDescRing] = {nullptr};
    int desc_i = 0;
    size_t desc_bytes = 0;
    // host staging for VSA_SRC_HOST planes (per stream, 2 slots)
    std::vector<uint8_t*> h_stage;
    std::vector<int64_t> h_stage_bytes;
    std::vector<hipEvent_t> stage_ev;
    // output drain
    uint64_t frames_read = 0, shots_read = 0;
    OutFrame* h_out_frames = nullptr;  // output rings in mapped pinned memory; the
    OutShot* h_out_shots = nullptr;    // decision kernel writes them through d_out_*
    uint64_t pushed_since_drain = 0;   // frames ingested after the newest published step
    // non-blocking publication: the decision kernel of each step writes the
    // output cursors into h_snap[step % kSnap] (mapped pinned memory, through
    // d_snap) and pub_ev of that slot is recorded after it
    PubSnap* h_snap = nullptr;
    PubSnap* d_snap = nullptr;
    hipEvent_t pub_ev[kSnap] = {};
    uint64_t pushed_cum[kSnap] = {};   // frames ingested up to and including each step
    uint64_t pushed_total = 0;
    int64_t pub_step = -1;             // newest step whose records are published
    // memory of closed streams, reusable once the device is past its last use
    struct PoolBlock { uint8_t* mem; uint64_t bytes; hipEvent_t ev; };
    std::vector<PoolBlock> pool;
    // pinned sources of the stream-ordered descriptor / state writes of open and close
    uint8_t* h_init = nullptr;
    size_t init_stride = 0;
    std::vector<hipEvent_t> init_ev;
    // per-kernel timing (profile = 1): a ring of event pairs per step
    int profile = 0;
    hipEvent_t prof_ev[kProfRing][kProfKinds][2] = {};
    int prof_used[kProfRing][kProfKinds] = {};
    int64_t prof_step = 0;
    int profile_every = 1;             // steps per timed step
    double prof_ms[kProfKinds] = {0};
    uint64_t prof_n[kProfKinds] = {0};
    int has8 = 0, has10 = 0;           // an open stream of that sample width (its launches run)
    int me_grid = 0;
    int cus = 256;
    // Motion-search launch autotuner.  The two motion-search launches of a
    // step share the GPU with the pyramids of the next step and the decisions
    // of the previous one, so a launch's own duration is not what to minimise:
    // a wider consecutive grid finishes sooner but starves the sparse pairs and
    // the decisions, which are the step's critical path.  Per size bucket
    // (log2 of the step's consecutive tiles) each candidate runs in turn for a
    // window of kTuneWindow live steps, timed between two events on the main
    // stream (the end of the step before the window, the end of its last
    // step), until each has kTuneSamples windows; the candidate with the
    // shortest window is kept (host-side hiccups only lengthen a window).
    int me_fixed = 0;                  // > 0: fixed workgroups per CU, no tuning
    bool no_intensity = false;         // skip the unary intensity measure
    struct TuneBucket { double ms[kTuneN] = {}; int n[kTuneN] = {}; int best = -1; };   // ms: shortest window
    TuneBucket tune[32];
    std::string tune_cache;            // the tuner's choices on disk (empty: none)
    struct TunePending { hipEvent_t ev0 = nullptr, ev1 = nullptr; int bucket = -1, cand = -1; };
    TunePending tune_ring[kTuneRing];
    int tune_head = 0;
    TunePending* tune_win = nullptr;   // the window in progress (its ev1 not yet recorded)
    int tune_left = 0;                 // steps left in it
    uint64_t counters[14] = {0};   // [10..13] host ns in vsa_step: descriptors, uploads, launches, total
};

namespace {

size_t desc_size(int max_streams) {
    return round_up(sizeof(StepStream) * max_streams, 256) + round_up(sizeof(int32_t) * max_streams, 256) +
           round_up(sizeof(PairTask) * max_streams, 256);
}

vsa_status ensure_partials(vsa_engine* e) {
    int64_t need = 0;
    for (const HostStream& s : e->streams)
        if (s.open) need += s.consec_tiles + s.sparse_tiles_max;
    if (need <= e->partials_cap) return VSA_OK;
    HIPCK(hipStreamSynchronize(e->stream_b), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream_c), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    // the new buffers first: if they do not fit, the old ones stay in place
    // and the open streams keep running
    const int64_t old_cap = e->partials_cap;
    const int64_t cap = std::max<int64_t>(need * 2, 4096);
    TilePartial* np = nullptr;
    int32_t *ncmap = nullptr, *nsmap = nullptr;
    // partials: consecutive pairs of even and odd steps, then the sparse pairs
    bool ok = hipMalloc(&np, sizeof(TilePartial) * cap * 3) == hipSuccess &&
              hipMalloc(&ncmap, sizeof(int32_t) * cap * (kAhead + 1)) == hipSuccess &&
              hipMalloc(&nsmap, sizeof(int32_t) * cap * 2) == hipSuccess;
    // the sparse tile maps planned by the last decision kernel are still to be
    // read by the next motion search: they move to the new allocation
    if (ok && e->d_smap) {
        for (int par = 0; ok && par < 2; ++par)
            ok = hipMemcpy(nsmap + par * cap, e->d_smap + par * old_cap, sizeof(int32_t) * old_cap,
                           hipMemcpyDeviceToDevice) == hipSuccess;
    }
    if (!ok) {
        for (void* q : {(void*)np, (void*)ncmap, (void*)nsmap})
            if (q) (void)hipFree(q);
        return fail(VSA_E_NOMEM, "tile partial buffer");
    }
    for (void* q : {(void*)e->d_partials, (void*)e->d_cmap, (void*)e->d_smap})
        if (q) (void)hipFree(q);
    e->d_partials = np;
    e->d_cmap = ncmap;
    e->d_smap = nsmap;
    e->partials_cap = cap;
    return VSA_OK;
}

// The dense flow's scratch for every open stream's pairs: a pair's starts at
// its tile prefix times the unit, in the list of its kind (consecutive or
// sparse); the unit is the largest any open stream needs.
vsa_status ensure_flow(vsa_engine* e) {
    if (e->params.search != 2) return VSA_OK;
    int64_t unit = 0, need_c = 0, need_s = 0;
    for (const HostStream& s : e->streams)
        if (s.open) {
            unit = std::max(unit, flow_unit(s.sd));
            need_c += s.consec_tiles;
            need_s += s.sparse_tiles_max;
        }
    if (unit <= e->flow_unit && need_c <= e->flow_tiles_c && need_s <= e->flow_tiles_s) return VSA_OK;
    HIPCK(hipStreamSynchronize(e->stream_b), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream_c), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    unit = std::max(unit, e->flow_unit);
    const int64_t tc = std::max(e->flow_tiles_c, need_c + need_c / 2);
    const int64_t ts = std::max(e->flow_tiles_s, need_s + need_s / 2);
    // the new buffers first: if they do not fit, the old ones stay in place
    uint8_t *nc = nullptr, *ns = nullptr;
    const bool ok = hipMalloc(&nc, (size_t)(unit * tc)) == hipSuccess &&
                    hipMalloc(&ns, (size_t)(unit * ts)) == hipSuccess;
    if (!ok) {
        if (nc) (void)hipFree(nc);
        return fail(VSA_E_NOMEM, "dense flow scratch");
    }
    if (e->d_flow_c) (void)hipFree(e->d_flow_c);
    if (e->d_flow_s) (void)hipFree(e->d_flow_s);
    e->d_flow_c = nc;
    e->d_flow_s = ns;
    e->flow_unit = unit;
    e->flow_tiles_c = tc;
    e->flow_tiles_s = ts;
    return VSA_OK;
}

// Tile histograms of one frame (written by each pyramid tile, summed by
// k_intensity).
int64_t tile_hist_bytes(const StreamDesc& sd, bool intensity) {
    if (!intensity) return 0;
    return round_up((int64_t)pyramid_tiles(sd) * (1 << sd.bits) * (int64_t)sizeof(uint16_t), 256);
}

uint64_t stream_bytes(const StreamDesc& sd, int64_t staging_pitch, bool intensity) {
    const int64_t info = round_up((int64_t)sizeof(FrameInfo) * sd.rs, 256);
    const int64_t mv = round_up((int64_t)sd.rs * sd.B_L * 2, 256);
    const int64_t stage = 2 * round_up(staging_pitch * sd.H, 256);
    return (uint64_t)(sd.slot_bytes * sd.rs + info + mv + tile_hist_bytes(sd, intensity) + stage);
}

// Add the elapsed time of a recorded event pair to the totals (stream already
// synchronised, or the pair is old enough to have completed).
void prof_collect(vsa_engine* e, int slot) {
    for (int k = 0; k < kProfKinds; ++k) {
        if (!e->prof_used[slot][k]) continue;
        float ms = 0.f;
        if (hipEventSynchronize(e->prof_ev[slot][k][1]) == hipSuccess &&
            hipEventElapsedTime(&ms, e->prof_ev[slot][k][0], e->prof_ev[slot][k][1]) == hipSuccess) {
            e->prof_ms[k] += ms;
            e->prof_n[k] += 1;
        }
        e->prof_used[slot][k] = 0;
    }
}

void prof_collect_all(vsa_engine* e) {
    if (!e->profile) return;
    for (int i = 0; i < kProfRing; ++i) prof_collect(e, i);
}

// Move the records up to the cursors c (all written by completed steps) from
// the mapped output rings into the per-stream queues.  Records of a stream
// closed since they were written carry an older epoch and are dropped.
vsa_status publish(vsa_engine* e, const PubSnap& c) {
    if (c.frames_written > e->frames_read) {
        if (c.frames_written - e->frames_read > kFramesCap) return fail(VSA_E_DEVICE, "frame ring overflow");
        for (uint64_t i = e->frames_read; i < c.frames_written; ++i) {
            const OutFrame& o = e->h_out_frames[i % kFramesCap];
            HostStream& s = e->streams[o.sid];
            if (!s.open || o.pad != s.epoch) continue;
            s.fq.push_back(o.r);
            s.frames_out += 1;
        }
        e->frames_read = c.frames_written;
    }
    if (c.shots_written > e->shots_read) {
        if (c.shots_written - e->shots_read > kShotsCap) return fail(VSA_E_DEVICE, "shot ring overflow");
        for (uint64_t i = e->shots_read; i < c.shots_written; ++i) {
            const OutShot& o = e->h_out_shots[i % kShotsCap];
            HostStream& s = e->streams[o.sid];
            if (!s.open || o.pad != s.epoch) continue;
            s.sq.push_back(o.r);
        }
        e->shots_read = c.shots_written;
    }
    for (HostStream& s : e->streams)
        if (s.open && s.ended && s.frames_out >= s.T_end) s.done = true;
    e->counters[6] = c.sparse_run;
    e->counters[9] = c.sparse_blocks;
    return VSA_OK;
}

// Wait for every queued step, then publish.
vsa_status drain(vsa_engine* e) {
    HIPCK(hipStreamSynchronize(e->stream_b), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream_c), "hipStreamSynchronize");
    HIPCK(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    DeviceCursors c;
    HIPCK(hipMemcpy(&c, e->d_cur, sizeof c, hipMemcpyDeviceToHost), "read cursors");
    const PubSnap ps{c.frames_written.v, c.shots_written.v, c.sparse_run.v, c.sparse_blocks.v};
    vsa_status st = publish(e, ps);
    if (st != VSA_OK) return st;
    e->pub_step = e->step_no - 1;
    e->pushed_since_drain = 0;
    prof_collect_all(e);
    return VSA_OK;
}

// Publish the steps the device has completed, without waiting.
vsa_status collect(vsa_engine* e) {
    int64_t s = e->pub_step + 1;
    while (s < e->step_no) {
        const hipError_t q = hipEventQuery(e->pub_ev[s % kSnap]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return hip_fail(q, "step completion query");
        ++s;
    }
    const int64_t last = s - 1;
    if (last <= e->pub_step) return VSA_OK;
    vsa_status st = publish(e, e->h_snap[last % kSnap]);
    if (st != VSA_OK) return st;
    e->pub_step = last;
    e->pushed_since_drain = e->pushed_total - e->pushed_cum[last % kSnap];
    return VSA_OK;
}

// Release a stream slot without waiting for the device: its descriptor is
// zeroed on the main stream (after every queued step that may read it) and
// its memory joins the pool once that point of the main stream is reached.
void free_stream(vsa_engine* e, int sid) {
    HostStream& s = e->streams[sid];
    hipEvent_t ev = nullptr;
    const uint8_t* zero = e->h_init + e->init_stride * (size_t)e->max_streams;
    bool ordered = hipMemcpyAsync(e->d_sds + sid, zero, sizeof(StreamDesc), hipMemcpyHostToDevice, e->stream) ==
                   hipSuccess;
    ordered = ordered && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(ev, e->stream) == hipSuccess;
    // the ingest stream may run ahead of the main stream: it must not see the
    // slot again before the zeroing
    ordered = ordered && hipStreamWaitEvent(e->stream_b, ev, 0) == hipSuccess;
    if (s.mem) {
        if (ordered) {
            e->pool.push_back({s.mem, s.mem_bytes, ev});
            ev = nullptr;
        } else {
            (void)hipStreamSynchronize(e->stream_b);
            (void)hipStreamSynchronize(e->stream_c);
            (void)hipStreamSynchronize(e->stream);
            (void)hipFree(s.mem);
        }
    }
    if (ev) (void)hipEventDestroy(ev);
    e->used -= s.bytes;
    s = HostStream();
}

// Device memory for a new stream: a pooled block of the same size whose last
// use has completed, else a fresh allocation (the pool is released first if
// that fails).
uint8_t* stream_alloc(vsa_engine* e, uint64_t bytes) {
    for (size_t i = 0; i < e->pool.size(); ++i) {
        auto& b = e->pool[i];
        if (b.bytes != bytes || hipEventQuery(b.ev) != hipSuccess) continue;
        uint8_t* m = b.mem;
        (void)hipEventDestroy(b.ev);
        e->pool.erase(e->pool.begin() + (long)i);
        return m;
    }
    uint8_t* m = nullptr;
    if (hipMalloc(&m, bytes) == hipSuccess) return m;
    (void)hipStreamSynchronize(e->stream_b);
    (void)hipStreamSynchronize(e->stream_c);
    (void)hipStreamSynchronize(e->stream);
    for (auto& b : e->pool) {
        (void)hipFree(b.mem);
        (void)hipEventDestroy(b.ev);
    }
    e->pool.clear();
    m = nullptr;
    if (hipMalloc(&m, bytes) == hipSuccess) return m;
    return nullptr;
}

void init_state(DecideState& st) {
    std::memset(&st, 0, sizeof st);
    st.t = 0;
    st.n = -1;
    st.T_end = -1;
    st.ss.open = 1;
    st.ss.phase = -1;
}

}  // namespace

extern "C" {

int32_t vsa_abi_version(void) { return VSA_ABI_VERSION; }

const char* vsa_last_error(void) { return g_err.c_str(); }

void vsa_default_params(vsa_params* p) {
    if (!p) return;
    p->block = 8; p->radius = 8; p->wmax = 512; p->lf_offset = 1; p->k_max = 4;
    p->a_static_fx = 64; p->w_hist = 8; p->n_ss = 20;
    p->a0 = 1.0; p->rho_f = 1.5; p->theta_f = 0.05; p->theta_f0 = 1.0; p->rho_d = 1.3; p->theta_d = 0.4;
    p->gamma = 0.5; p->tau_c = 0.65; p->eps = 0.2; p->tau_p = 2.0; p->theta_kf = 3.0;
    p->search = 0; p->refine = 1;
}

static void tune_cache_load(vsa_engine* e);

vsa_status vsa_params_from_json(const char* json, vsa_params* out) {
    if (!json || !out) return fail(VSA_E_INVAL, "NULL argument");
    vsa_params p;
    vsa_default_params(&p);
    struct IntField { const char* name; int32_t* v; };
    struct DblField { const char* name; double* v; };
    const IntField ints[] = {{"block", &p.block}, {"radius", &p.radius}, {"wmax", &p.wmax},
                             {"lf_offset", &p.lf_offset}, {"k_max", &p.k_max}, {"a_static_fx", &p.a_static_fx},
                             {"w_hist", &p.w_hist}, {"n_ss", &p.n_ss}, {"search", &p.search}, {"refine", &p.refine}};
    const DblField dbls[] = {{"a0", &p.a0}, {"rho_f", &p.rho_f}, {"theta_f", &p.theta_f},
                             {"theta_f0", &p.theta_f0}, {"rho_d", &p.rho_d}, {"theta_d", &p.theta_d},
                             {"gamma", &p.gamma}, {"tau_c", &p.tau_c}, {"eps", &p.eps}, {"tau_p", &p.tau_p},
                             {"theta_kf", &p.theta_kf}};
    const char* c = json;
    auto ws = [&]() { while (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r') ++c; };
    ws();
    if (*c++ != '{') return fail(VSA_E_INVAL, "params JSON: expected '{'");
    ws();
    if (*c == '}') { ++c; ws(); if (*c) return fail(VSA_E_INVAL, "params JSON: text after the object"); *out = p; return VSA_OK; }
    for (;;) {
        ws();
        if (*c++ != '"') return fail(VSA_E_INVAL, "params JSON: expected a key");
        const char* k0 = c;
        while (*c && *c != '"') ++c;
        if (!*c) return fail(VSA_E_INVAL, "params JSON: unterminated key");
        const std::string key(k0, c - k0);
        ++c;
        ws();
        if (*c++ != ':') return fail(VSA_E_INVAL, "params JSON: expected ':'");
        ws();
        char* end = nullptr;
        const double v = std::strtod(c, &end);
        if (end == c) return fail(VSA_E_INVAL, "params JSON: expected a number");
        const std::string lit(c, end - c);
        c = end;
        // JSON numbers only: no infinities, NaN or hexadecimal forms
        if (!std::isfinite(v) || lit.find_first_of("xXnNiI") != std::string::npos)
            return fail(VSA_E_INVAL, "params JSON: " + key + " is not a finite JSON number");
        bool found = false;
        for (const IntField& f : ints)
            if (key == f.name) {
                if (lit.find_first_of(".eE") != std::string::npos || v < -2147483648.0 || v > 2147483647.0)
                    return fail(VSA_E_INVAL, "params JSON: " + key + " must be an int32");
                *f.v = (int32_t)v;
                found = true;
            }
        for (const DblField& f : dbls)
            if (key == f.name) { *f.v = v; found = true; }
        if (!found) return fail(VSA_E_INVAL, "params JSON: unknown key " + key);
        ws();
        if (*c == ',') { ++c; continue; }
        if (*c == '}') { ++c; break; }
        return fail(VSA_E_INVAL, "params JSON: expected ',' or '}'");
    }
    ws();
    if (*c) return fail(VSA_E_INVAL, "params JSON: text after the object");
    *out = p;
    return VSA_OK;
}

vsa_status vsa_engine_create(const vsa_engine_config* cfg, vsa_engine** out) {
    if (!cfg || !out) return fail(VSA_E_INVAL, "NULL argument");
    *out = nullptr;
    if (cfg->max_streams < 1 || cfg->max_streams > kMaxStreams)
        return fail(VSA_E_INVAL, "max_streams must be in 1..1024");
    if (cfg->schedule != VSA_SCHEDULE_SPARSE && cfg->schedule != VSA_SCHEDULE_DENSE)
        return fail(VSA_E_INVAL, "unknown schedule");
    if (cfg->use_graph)
        return fail(VSA_E_UNSUPPORTED, "use_graph: a captured step graph costs more host time per replay than "
                                       "its direct launches");
    if (cfg->me_wgs_per_cu < 0 || cfg->me_wgs_per_cu > 8)
        return fail(VSA_E_INVAL, "me_wgs_per_cu must be in 0..8");
    vsa_params p;
    if (cfg->params_json) {
        const vsa_status sj = vsa_params_from_json(cfg->params_json, &p);
        if (sj != VSA_OK) return sj;
    } else if (cfg->params) {
        p = *cfg->params;
    } else {
        vsa_default_params(&p);
    }
    vsa_status st = check_params(p);
    if (st != VSA_OK) return st;
    int ndev = 0;
    HIPCK(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (cfg->device < 0 || cfg->device >= ndev) return fail(VSA_E_INVAL, "no such device");
    HIPCK(hipSetDevice(cfg->device), "hipSetDevice");
    vsa_engine* e = new vsa_engine();
    e->device = cfg->device;
    e->params = p;
    e->schedule = cfg->schedule;
    e->dp = decide_params(p, cfg->schedule == VSA_SCHEDULE_DENSE);
    e->max_streams = cfg->max_streams;
    e->debug_log = cfg->debug_log;
    e->streams.resize(cfg->max_streams);
    e->slot_epoch.assign(cfg->max_streams, 0);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    e->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
    e->cus = cus;
    e->me_grid = cus * 8;
    e->me_fixed = cfg->me_wgs_per_cu;
    e->no_intensity = cfg->no_intensity != 0;
    if (cfg->autotune_cache) {
        e->tune_cache = cfg->autotune_cache;
        tune_cache_load(e);
    }
    const int M = cfg->max_streams;
    auto dalloc = [&](void** p_, size_t n) { return hipMalloc(p_, n) == hipSuccess; };
    bool ok = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&e->stream_b, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&e->stream_c, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i <= kAhead; ++i)
        ok = hipEventCreateWithFlags(&e->ev_a[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&e->ev_b[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&e->ev_c[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&e->ev_h[i], hipEventDisableTiming) == hipSuccess;
    ok = ok && dalloc((void**)&e->d_sds, sizeof(StreamDesc) * M);
    ok = ok && dalloc((void**)&e->d_states, sizeof(DecideState) * M);
    ok = ok && dalloc((void**)&e->d_closed, sizeof(vsa_shot_result) * kMaxClosed * M);
    ok = ok && dalloc((void**)&e->d_results, sizeof(PairResult) * M * kResSlots);
    ok = ok && dalloc((void**)&e->d_sparse, 2 * sizeof(PairTask) * M * kMaxTasksPerStream);
    ok = ok && dalloc((void**)&e->d_sjobs, 2 * sizeof(TileJob) * M * kMaxTasksPerStream);
    ok = ok && dalloc((void**)&e->d_cjobs, (kAhead + 1) * sizeof(TileJob) * M);
    ok = ok && dalloc((void**)&e->d_cur, sizeof(DeviceCursors));
    e->desc_bytes = desc_size(M);
    e->desc_build.assign(e->desc_bytes, 0);
    ok = ok && dalloc((void**)&e->d_desc, (kAhead + 1) * e->desc_bytes);
    for (int i = 0; ok && i < kDescRing; ++i) {
        ok = hipHostMalloc((void**)&e->h_desc[i], e->desc_bytes, hipHostMallocMapped) == hipSuccess &&
             hipHostGetDevicePointer(&e->h_desc_dev[i], e->h_desc[i], 0) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&e->desc_ev[i], hipEventDisableTiming) == hipSuccess;
    }
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    ok = ok && hipHostMalloc((void**)&e->h_out_frames, sizeof(OutFrame) * kFramesCap, mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&e->d_out_frames, e->h_out_frames, 0) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&e->h_out_shots, sizeof(OutShot) * kShotsCap, mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&e->d_out_shots, e->h_out_shots, 0) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&e->h_snap, sizeof(PubSnap) * kSnap, mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&e->d_snap, e->h_snap, 0) == hipSuccess;
    for (int i = 0; ok && i < kSnap; ++i)
        ok = hipEventCreateWithFlags(&e->pub_ev[i], hipEventDisableTiming) == hipSuccess;
    for (auto& t : e->tune_ring)
        ok = ok && hipEventCreate(&t.ev0) == hipSuccess && hipEventCreate(&t.ev1) == hipSuccess;
    e->init_stride = round_up(sizeof(StreamDesc) + sizeof(DecideState), 256);
    ok = ok && hipHostMalloc((void**)&e->h_init, e->init_stride * (M + 1), hipHostMallocDefault) == hipSuccess;
    if (ok) std::memset(e->h_init, 0, e->init_stride * (M + 1));   // the last entry stays zero
    e->init_ev.assign(M, nullptr);
    for (int i = 0; ok && i < M; ++i)
        ok = hipEventCreateWithFlags(&e->init_ev[i], hipEventDisableTiming) == hipSuccess;
    if (ok && e->debug_log) ok = dalloc((void**)&e->d_log, sizeof(int32_t) * 6 * kLogCapPerStream * M);
    if (ok) {
        ok = hipMemset(e->d_sds, 0, sizeof(StreamDesc) * M) == hipSuccess &&
             hipMemset(e->d_cur, 0, sizeof(DeviceCursors)) == hipSuccess &&
             hipMemset(e->d_results, 0, sizeof(PairResult) * M * kResSlots) == hipSuccess;
    }
    e->profile = cfg->profile < 0 ? 0 : (cfg->profile > 2 ? 2 : cfg->profile);
    e->profile_every = cfg->profile_every > 1 ? cfg->profile_every : 1;
    for (int i = 0; ok && e->profile && i < kProfRing; ++i)
        for (int k = 0; ok && k < kProfKinds; ++k)
            for (int j = 0; ok && j < 2; ++j)
                ok = hipEventCreate(&e->prof_ev[i][k][j]) == hipSuccess;
    e->h_stage.assign(2 * M, nullptr);
    e->h_stage_bytes.assign(2 * M, 0);
    e->stage_ev.assign(2 * M, nullptr);
    if (!ok) {
        vsa_engine_destroy(e);
        return fail(VSA_E_NOMEM, "engine allocation failed");
    }
    *out = e;
    return VSA_OK;
}

void vsa_engine_destroy(vsa_engine* e) {
    if (!e) return;
    (void)hipSetDevice(e->device);
    if (e->stream_b) (void)hipStreamSynchronize(e->stream_b);
    if (e->stream_c) (void)hipStreamSynchronize(e->stream_c);
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    for (size_t i = 0; i < e->streams.size(); ++i)
        if (e->streams[i].mem) (void)hipFree(e->streams[i].mem);
    for (const auto& b : e->pool) {
        (void)hipFree(b.mem);
        if (b.ev) (void)hipEventDestroy(b.ev);
    }
    for (hipEvent_t ev : e->init_ev) if (ev) (void)hipEventDestroy(ev);
    if (e->h_init) (void)hipHostFree(e->h_init);
    for (int i = 0; i < kSnap; ++i) if (e->pub_ev[i]) (void)hipEventDestroy(e->pub_ev[i]);
    for (auto& t : e->tune_ring) {
        if (t.ev0) (void)hipEventDestroy(t.ev0);
        if (t.ev1) (void)hipEventDestroy(t.ev1);
    }
    if (e->h_snap) (void)hipHostFree(e->h_snap);
    for (uint8_t* h : e->h_stage) if (h) (void)hipHostFree(h);
    for (hipEvent_t ev : e->stage_ev) if (ev) (void)hipEventDestroy(ev);
    void* dev[] = {e->d_sds, e->d_states, e->d_closed, e->d_results, e->d_sparse, e->d_cur,
                   e->d_partials, e->d_log, e->d_desc, e->d_sjobs, e->d_cjobs, e->d_cmap, e->d_smap,
                   e->d_flow_c, e->d_flow_s};
    for (void* p : dev) if (p) (void)hipFree(p);
    for (int i = 0; i < kDescRing; ++i) {
        if (e->h_desc[i]) (void)hipHostFree(e->h_desc[i]);
        if (e->desc_ev[i]) (void)hipEventDestroy(e->desc_ev[i]);
    }
    if (e->h_out_frames) (void)hipHostFree(e->h_out_frames);
    if (e->h_out_shots) (void)hipHostFree(e->h_out_shots);
    for (int i = 0; i < kProfRing; ++i)
        for (int k = 0; k < kProfKinds; ++k)
            for (int j = 0; j < 2; ++j)
                if (e->prof_ev[i][k][j]) (void)hipEventDestroy(e->prof_ev[i][k][j]);
    for (int i = 0; i <= kAhead; ++i) {
        if (e->ev_a[i]) (void)hipEventDestroy(e->ev_a[i]);
        if (e->ev_b[i]) (void)hipEventDestroy(e->ev_b[i]);
        if (e->ev_c[i]) (void)hipEventDestroy(e->ev_c[i]);
        if (e->ev_h[i]) (void)hipEventDestroy(e->ev_h[i]);
    }
    if (e->stream_c) (void)hipStreamDestroy(e->stream_c);
    if (e->stream_b) (void)hipStreamDestroy(e->stream_b);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

static vsa_status prepare_stream(const vsa_engine* e, const vsa_stream_desc* d, StreamDesc& sd, Geo& g,
                                 int64_t& staging_pitch, uint64_t& bytes) {
    if (!d) return fail(VSA_E_INVAL, "NULL stream description");
    if (d->bit_depth != 8 && d->bit_depth != 10) return fail(VSA_E_INVAL, "bit_depth must be 8 or 10");
    const int kmax = d->k_max ? d->k_max : e->params.k_max;
    if (kmax < 1 || kmax > kMaxKmax) return fail(VSA_E_INVAL, "k_max must be in 1..15");
    vsa_status st = make_geo(d->width, d->height, e->params, kmax, g);
    if (st != VSA_OK) return st;
    layout(g, d->width, d->height, d->bit_depth, kmax, sd);
    sd.search = e->params.search;
    if (sd.search == 2 && (int64_t)d->width * d->height >= (1ll << 31))
        return fail(VSA_E_UNSUPPORTED, "frames of 2^31 samples or more with the dense flow");
    st = check_exact_sums(sd);
    if (st != VSA_OK) return st;
    staging_pitch = round_up((int64_t)d->width * (d->bit_depth == 8 ? 1 : 2), 256);
    bytes = stream_bytes(sd, staging_pitch, !e->no_intensity);
    return VSA_OK;
}

uint64_t vsa_stream_footprint(const vsa_engine* e, const vsa_stream_desc* d) {
    if (!e) return 0;
    StreamDesc sd;
    Geo g;
    int64_t sp;
    uint64_t bytes;
    if (prepare_stream(e, d, sd, g, sp, bytes) != VSA_OK) return 0;
    return bytes + stream_tile_bytes(sd);
}

vsa_status vsa_stream_open(vsa_engine* e, const vsa_stream_desc* d, int32_t* sid) {
    if (!e || !sid) return fail(VSA_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(e->mu);
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    StreamDesc sd;
    Geo g;
    int64_t sp;
    uint64_t bytes;
    vsa_status st = prepare_stream(e, d, sd, g, sp, bytes);
    if (st != VSA_OK) return st;
    int slot = -1;
    for (int i = 0; i < e->max_streams; ++i)
        if (!e->streams[i].open) { slot = i; break; }
    const uint64_t part = stream_tile_bytes(sd);
    if (slot < 0 || e->used + bytes + part > e->budget) {
        e->counters[3] += 1;
        return fail(VSA_E_ADMIT, slot < 0 ? "no free stream slot" : "HBM budget exhausted");
    }
    HostStream& s = e->streams[slot];
    const int epoch = e->slot_epoch[slot] + 1;
    e->slot_epoch[slot] = epoch;
    sd.epoch = epoch;
    uint8_t* mem = stream_alloc(e, bytes);
    if (!mem) {
        e->counters[3] += 1;
        return fail(VSA_E_ADMIT, "device allocation for the stream failed");
    }
    int64_t off = sd.slot_bytes * sd.rs;
    sd.ring = mem;
    sd.info = reinterpret_cast<FrameInfo*>(mem + off);
    off += round_up((int64_t)sizeof(FrameInfo) * sd.rs, 256);
    sd.mv = reinterpret_cast<int8_t*>(mem + off);
    off += round_up((int64_t)sd.rs * sd.B_L * 2, 256);
    sd.tileh = e->no_intensity ? nullptr : reinterpret_cast<uint16_t*>(mem + off);
    off += tile_hist_bytes(sd, !e->no_intensity);
    s = HostStream();
    s.open = true;
    s.desc = *d;
    s.sd = sd;
    s.geo = g;
    s.mem = mem;
    s.mem_bytes = bytes;
    s.bytes = bytes + part;
    s.staging_pitch = sp;
    s.staging_dev[0] = mem + off;
    s.staging_dev[1] = mem + off + round_up(sp * sd.H, 256);
    s.consec_tiles = frame_pair_tiles(sd.search, sd.wl[0], sd.hl[0]);
    s.sparse_tiles_max = max_sparse_tiles(sd);
    s.epoch = epoch;
    e->used += s.bytes;
    // descriptor, decision state and frame records are initialised on the
    // main stream, after every queued step (which may still use this slot's
    // previous stream); the ingest stream waits for it before its next step
    DecideState ds;
    init_state(ds);
    uint8_t* src = e->h_init + e->init_stride * (size_t)slot;
    hipError_t err = hipEventSynchronize(e->init_ev[slot]);   // the previous open's copies
    if (err == hipSuccess) {
        std::memcpy(src, &sd, sizeof sd);
        std::memcpy(src + sizeof(StreamDesc), &ds, sizeof ds);
        err = hipMemcpyAsync(e->d_sds + slot, src, sizeof sd, hipMemcpyHostToDevice, e->stream);
    }
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->d_states + slot, src + sizeof(StreamDesc), sizeof ds, hipMemcpyHostToDevice,
                             e->stream);
    if (err == hipSuccess) err = hipMemsetAsync(sd.info, 0, sizeof(FrameInfo) * sd.rs, e->stream);
    if (err == hipSuccess) err = hipEventRecord(e->init_ev[slot], e->stream);
    if (err == hipSuccess) err = hipStreamWaitEvent(e->stream_b, e->init_ev[slot], 0);
    if (err != hipSuccess) { free_stream(e, slot); return hip_fail(err, "stream init"); }
    st = ensure_partials(e);
    if (st == VSA_OK) st = ensure_flow(e);
    if (st != VSA_OK) { free_stream(e, slot); return st; }
    if (sd.bits == 10) e->has10 = 1;
    else e->has8 = 1;
    e->counters[2] += 1;
    *sid = slot;
    return VSA_OK;
}

static HostStream* get_stream(vsa_engine* e, int32_t sid) {
    if (!e || sid < 0 || sid >= e->max_streams || !e->streams[sid].open) return nullptr;
    return &e->streams[sid];
}

vsa_status vsa_stream_push(vsa_engine* e, int32_t sid, const void* luma, int64_t pitch, int32_t src, int64_t pts) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    if (!luma) return fail(VSA_E_INVAL, "NULL plane");
    const int64_t row = (int64_t)s->sd.W * (s->sd.bits == 8 ? 1 : 2);
    if (pitch < row) return fail(VSA_E_INVAL, "pitch smaller than a row");
    if (s->ended) return fail(VSA_E_STATE, "push after end of stream");
    if (s->pending) return fail(VSA_E_AGAIN, "a frame is already waiting for a step");
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    const int slot = s->next_frame & 1;
    if (src == VSA_SRC_HOST) {
        const int k = 2 * sid + slot;
        const int64_t need = s->staging_pitch * s->sd.H;
        if (e->stage_ev[k]) HIPCK(hipEventSynchronize(e->stage_ev[k]), "staging reuse");
        else HIPCK(hipEventCreateWithFlags(&e->stage_ev[k], hipEventDisableTiming), "event");
        if (e->h_stage_bytes[k] < need) {   // a slot may be reused by a larger format
            if (e->h_stage[k]) HIPCK(hipHostFree(e->h_stage[k]), "pinned staging");
            e->h_stage[k] = nullptr;
            e->h_stage_bytes[k] = 0;
            HIPCK(hipHostMalloc((void**)&e->h_stage[k], need, hipHostMallocDefault), "pinned staging");
            e->h_stage_bytes[k] = need;
        }
        const uint8_t* p = static_cast<const uint8_t*>(luma);
        for (int y = 0; y < s->sd.H; ++y) std::memcpy(e->h_stage[k] + y * s->staging_pitch, p + y * pitch, row);
        if (s->sd.bits == 10 && !samples_10bit_ok(e->h_stage[k], s->staging_pitch, s->sd.W, s->sd.H))
            return fail(VSA_E_INVAL, "10-bit plane holds a sample above 1023");
        s->pend_src = e->h_stage[k];
        s->pend_pitch = s->staging_pitch;
    } else if (src == VSA_SRC_DEVICE_COPY) {
        HIPCK(hipMemcpy2DAsync(s->staging_dev[slot], s->staging_pitch, luma, pitch, row, s->sd.H,
                               hipMemcpyDeviceToDevice, e->stream_b), "device copy");
        HIPCK(hipStreamSynchronize(e->stream_b), "device copy");
        s->pend_src = s->staging_dev[slot];
        s->pend_pitch = s->staging_pitch;
    } else if (src == VSA_SRC_DEVICE_BORROW || src == VSA_SRC_HOST_BORROW) {
        s->pend_src = luma;
        s->pend_pitch = pitch;
    } else {
        return fail(VSA_E_INVAL, "unknown source kind");
    }
    s->pend_mode = src;
    s->pend_pts = pts;
    s->pending = true;
    return VSA_OK;
}

vsa_status vsa_stream_push_batch(vsa_engine* e, int32_t n, const int32_t* sids, const void* const* planes,
                                 const int64_t* pitches, int32_t src, const int64_t* pts, int32_t* status) {
    if (!e || n < 0 || (n > 0 && (!sids || !planes || !pitches))) return fail(VSA_E_INVAL, "bad argument");
    vsa_status first = VSA_OK;
    for (int32_t i = 0; i < n; ++i) {
        const vsa_status st = vsa_stream_push(e, sids[i], planes[i], pitches[i], src, pts ? pts[i] : 0);
        if (status) status[i] = st;
        if (st != VSA_OK && first == VSA_OK) first = st;
    }
    return first;
}

vsa_status vsa_engine_kernel_times(vsa_engine* e, double* ms, uint64_t* launches, int32_t reset) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    if (!e->profile) return fail(VSA_E_STATE, "engine created without profile");
    for (int k = 0; k < kProfKinds; ++k) {
        if (ms) ms[k] = e->prof_ms[k];
        if (launches) launches[k] = e->prof_n[k];
        if (reset) { e->prof_ms[k] = 0.0; e->prof_n[k] = 0; }
    }
    return VSA_OK;
}

vsa_status vsa_stream_end(vsa_engine* e, int32_t sid) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    if (s->ended) return fail(VSA_E_STATE, "stream already ended");
    s->ended = true;
    s->T_end = s->next_frame + (s->pending ? 1 : 0);
    if (s->T_end == 0) s->done = true;
    return VSA_OK;
}

int32_t vsa_stream_done(vsa_engine* e, int32_t sid) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    return s->done ? 1 : 0;
}

static inline uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The tuner's cache file: one line per settled bucket, "cus S search S bucket
// B consec C sparse P" (workgroups per CU of the two grids).  A line counts
// only for this device's CU count and search mode, and only if its pair is
// one of the candidates; later lines win.
static void tune_cache_load(vsa_engine* e) {
    FILE* f = std::fopen(e->tune_cache.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int cus = 0, search = 0, bucket = -1, consec = 0, sparse = 0;
        if (std::sscanf(line, "cus %d search %d bucket %d consec %d sparse %d", &cus, &search, &bucket, &consec,
                        &sparse) != 5)
            continue;
        if (cus != e->cus || search != e->params.search || bucket < 0 || bucket >= 32) continue;
        for (int c = 0; c < kTuneN; ++c)
            if (kTuneCands[c].consec == consec && kTuneCands[c].sparse == sparse) e->tune[bucket].best = c;
    }
    std::fclose(f);
}

static void tune_cache_store(vsa_engine* e, int bucket, int cand) {
    if (e->tune_cache.empty()) return;
    FILE* f = std::fopen(e->tune_cache.c_str(), "a");
    if (!f) return;   // the cache only saves tuning time
    std::fprintf(f, "cus %d search %d bucket %d consec %d sparse %d\n", e->cus, e->params.search, bucket,
                 kTuneCands[cand].consec, kTuneCands[cand].sparse);
    std::fclose(f);
}

// Add a finished window to its bucket; once every candidate has kTuneSamples
// windows the bucket keeps the fastest.  With wait, block for the timing.
void tune_harvest(vsa_engine* e, vsa_engine::TunePending& t, bool wait) {
    if (t.bucket < 0 || &t == e->tune_win) return;
    if (!wait && hipEventQuery(t.ev1) != hipSuccess) return;
    if (wait) (void)hipEventSynchronize(t.ev1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev0, t.ev1) == hipSuccess) {
        auto& b = e->tune[t.bucket];
        if (b.best < 0) {
            b.ms[t.cand] = b.n[t.cand] ? std::min<double>(b.ms[t.cand], ms) : ms;
            b.n[t.cand] += 1;
            bool all = true;
            for (int c = 0; c < kTuneN; ++c) all = all && b.n[c] >= kTuneSamples;
            if (all) {
                int best = 0;
                for (int c = 1; c < kTuneN; ++c)
                    if (b.ms[c] < b.ms[best]) best = c;
                b.best = best;
                tune_cache_store(e, t.bucket, best);
            }
        }
    }
    t.bucket = -1;
}

// Candidate for the next motion-search window: the bucket's choice once
// tuned, else the candidate with the fewest windows (finished windows of
// earlier steps are collected first, without waiting).
int me_candidate(vsa_engine* e, int bucket) {
    if (e->me_fixed) return 0;
    for (auto& t : e->tune_ring) tune_harvest(e, t, false);
    auto& b = e->tune[bucket];
    if (b.best >= 0) return b.best;
    int n[kTuneN];                     // windows per candidate, finished or in flight
    for (int k = 0; k < kTuneN; ++k) n[k] = b.n[k];
    for (const auto& t : e->tune_ring) if (t.bucket == bucket) n[t.cand] += 1;
    int c = 0;
    for (int k = 1; k < kTuneN; ++k) if (n[k] < n[c]) c = k;
    return c;
}

vsa_status vsa_step(vsa_engine* e, void* hip_stream) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    const uint64_t t_start = now_ns();
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    hipStream_t user = static_cast<hipStream_t>(hip_stream);
    // bound the output produced between syncs by the ring capacities
    // A stream emits, between two drains, at most the frames it ingested plus
    // the backlog it held (< rs) plus one; shots never outnumber frames + 3.
    uint64_t backlog = 0, step_push = 0;
    int n_open = 0;
    for (const HostStream& s : e->streams)
        if (s.open && !s.done) { backlog += s.sd.rs + 4; step_push += s.pending ? 1 : 0; ++n_open; }
    if (n_open == 0) return VSA_OK;
    if (e->pushed_since_drain + step_push + backlog > std::min(kFramesCap, kShotsCap)) {
        vsa_status st = collect(e);
        if (st == VSA_OK && e->pushed_since_drain + step_push + backlog > std::min(kFramesCap, kShotsCap))
            st = drain(e);
        if (st != VSA_OK) return st;
    }
    const int ps = (int)(e->prof_step % kProfRing);
    if (e->profile) prof_collect(e, ps);
    // profile 1: the pyramid and motion-search launches only; 2: every kernel.
    // Kernels are timed by events stamped from their own dispatch (the first
    // launch of a kind starts the pair, the last one stops it); the whole step
    // by recorded events.
    const bool prof_now = e->profile && (e->step_no % e->profile_every) == 0;
    auto profiled = [&](int k) { return prof_now && !(e->profile == 1 && k > 3); };
    auto timing = [&](int k, bool first, bool last) {
        LaunchTiming t;
        if (!profiled(k)) return t;
        if (first) t.start = e->prof_ev[ps][k][0];
        if (last) {
            t.stop = e->prof_ev[ps][k][1];
            e->prof_used[ps][k] = 1;
        }
        return t;
    };
    auto prof = [&](int k, int j, hipStream_t st) {
        if (!profiled(k)) return;
        (void)hipEventRecord(e->prof_ev[ps][k][j], st);
        if (j == 1) e->prof_used[ps][k] = 1;
    };
    const int par = (int)(e->step_no & 1);
    const int slot_s = (int)(e->step_no % (kAhead + 1));
    hipStream_t A = e->stream, Bs = e->stream_b;
    // the ingest stream never runs more than kAhead steps ahead of the main
    // stream: before step s it waits for the main stream's step s - kAhead - 1
    // (recorded in the same event slot)
    HIPCK(hipStreamWaitEvent(Bs, e->ev_a[slot_s], 0), "wait");
    // step descriptor in a pinned ring slot
    const int di = e->desc_i;
    e->desc_i = (e->desc_i + 1) % kDescRing;
    uint8_t* h = e->desc_build.data();
    const int M = e->max_streams;
    StepStream* steps = reinterpret_cast<StepStream*>(h);
    int32_t* k1 = reinterpret_cast<int32_t*>(h + round_up(sizeof(StepStream) * M, 256));
    PairTask* consec = reinterpret_cast<PairTask*>(h + round_up(sizeof(StepStream) * M, 256) +
                                                    round_up(sizeof(int32_t) * M, 256));
    int n_steps = 0, n_k1 = 0, n_consec = 0, consec_tiles = 0;
    for (int sid = 0; sid < M; ++sid) {
        HostStream& s = e->streams[sid];
        if (!s.open || s.done) continue;
        StepStream& ss = steps[n_steps];
        std::memset(&ss, 0, sizeof ss);
        ss.sid = sid;
        ss.has_frame = s.pending ? 1 : 0;
        ss.frame = s.pending ? s.next_frame : -1;
        ss.ended_T = s.ended ? s.T_end : -1;
        ss.pts = s.pend_pts;
        if (s.pending) {
            const int slot = s.next_frame & 1;
            if (s.pend_mode == VSA_SRC_HOST) {
                HIPCK(hipMemcpyAsync(s.staging_dev[slot], s.pend_src, s.staging_pitch * s.sd.H,
                                     hipMemcpyHostToDevice, Bs), "plane upload");
                HIPCK(hipEventRecord(e->stage_ev[2 * sid + slot], Bs), "event");
                ss.src = s.staging_dev[slot];
                ss.src_pitch = s.pend_pitch;
            } else if (s.pend_mode == VSA_SRC_HOST_BORROW) {
                // the caller's (pinned) plane straight into the device staging slot
                const int64_t row = (int64_t)s.sd.W * (s.sd.bits == 8 ? 1 : 2);
                HIPCK(hipMemcpy2DAsync(s.staging_dev[slot], s.staging_pitch, s.pend_src, s.pend_pitch, row,
                                       s.sd.H, hipMemcpyHostToDevice, Bs), "plane upload");
                ss.src = s.staging_dev[slot];
                ss.src_pitch = s.staging_pitch;
            } else {
                ss.src = s.pend_src;
                ss.src_pitch = s.pend_pitch;
            }
            ss.k1_tiles = pyramid_tiles(s.sd);
            k1[n_k1++] = n_steps;
            if (s.next_frame >= 1) {
                PairTask& t = consec[n_consec++];
                std::memset(&t, 0, sizeof t);
                t.sid = sid;
                t.kind = MK_CONSEC;
                t.ref = s.next_frame - 1;
                t.oth = s.next_frame;
                t.ref_field = t.oth_field = PL_FRAME;
                t.level = s.sd.L;
                t.result = -1;
                t.tiles = s.consec_tiles;
                t.tile_prefix = consec_tiles;
                t.flags = TF_MV_RING;
                t.epoch = s.sd.epoch;
                consec_tiles += t.tiles;
                ss.consec_tiles = t.tiles;
                ss.consec_prefix = t.tile_prefix;
            }
        }
        ++n_steps;
    }
    // group the pyramid work by (sample width, working level): one launch per group
    struct K1Group { int bits, L, first, count, tiles; };
    K1Group groups[10];
    int n_groups = 0;
    {
        std::stable_sort(k1, k1 + n_k1, [&](int a, int b) {
            const StreamDesc& sa = e->streams[steps[a].sid].sd;
            const StreamDesc& sb = e->streams[steps[b].sid].sd;
            return sa.bits * 8 + sa.L < sb.bits * 8 + sb.L;
        });
        for (int i = 0; i < n_k1; ++i) {
            StepStream& ss = steps[k1[i]];
            const StreamDesc& sd = e->streams[ss.sid].sd;
            if (n_groups == 0 || groups[n_groups - 1].bits != sd.bits || groups[n_groups - 1].L != sd.L)
                groups[n_groups++] = K1Group{sd.bits, sd.L, i, 0, 0};
            K1Group& gr = groups[n_groups - 1];
            ss.k1_prefix = gr.tiles;
            gr.tiles += ss.k1_tiles;
            gr.count += 1;
        }
    }
    const size_t off_k1 = round_up(sizeof(StepStream) * M, 256);
    const size_t off_consec = off_k1 + round_up(sizeof(int32_t) * M, 256);
    const uint64_t t_built = now_ns();
    if (user) {
        hipEvent_t ev;
        HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
        HIPCK(hipEventRecord(ev, user), "event");
        HIPCK(hipStreamWaitEvent(Bs, ev, 0), "wait");
        HIPCK(hipStreamWaitEvent(e->stream_c, ev, 0), "wait");
        HIPCK(hipStreamWaitEvent(A, ev, 0), "wait");
        (void)hipEventDestroy(ev);
    }
    uint8_t* ddesc = e->d_desc + (size_t)slot_s * e->desc_bytes;
    prof(5, 0, Bs);
    {
        // one sequential write into the pinned slot (after the device has read
        // its previous contents), then a copy kernel on the ingest stream
        const size_t used = off_consec + sizeof(PairTask) * std::max(n_consec, 1);
        HIPCK(hipEventSynchronize(e->desc_ev[di]), "descriptor reuse");
        std::memcpy(e->h_desc[di], h, used);
        HIPCK(launch_copy16(e->h_desc_dev[di], ddesc, (int64_t)used, Bs), "descriptor upload");
    }
    HIPCK(hipEventRecord(e->desc_ev[di], Bs), "event");
    const uint64_t t_upload = now_ns();
    const StepStream* d_steps = reinterpret_cast<const StepStream*>(ddesc);
    TileJob* cjobs = e->d_cjobs + (size_t)slot_s * M;
    int32_t* cmap = e->d_cmap + (size_t)slot_s * e->partials_cap;
    const int32_t* d_k1 = reinterpret_cast<const int32_t*>(ddesc + off_k1);
    if (n_k1 > 0) {
        for (int gi = 0; gi < n_groups; ++gi) {
            const K1Group& gr = groups[gi];
            HIPCK(launch_pyramid(gr.bits, gr.L, e->d_sds, d_steps, d_k1 + gr.first, gr.count, gr.tiles, cjobs, cmap,
                                 Bs, timing(0, gi == 0, gi == n_groups - 1)),
                  "pyramid launch");
        }
    }
    HIPCK(hipEventRecord(e->ev_b[slot_s], Bs), "event");
    // the frames' intensity measures from the tile histograms: off the search
    // stream's path; the decisions (which may emit this step's records) wait
    if (!e->no_intensity) {
        HIPCK(launch_intensity(e->d_sds, d_steps, d_k1, n_k1, Bs), "intensity launch");
        HIPCK(hipEventRecord(e->ev_h[slot_s], Bs), "event");
    }
    // Consecutive pairs run on the search stream C once this step's pyramids
    // are done and the decisions of step s-2 (which read the consecutive
    // partials of this parity) have finished, so they overlap the decisions
    // of step s-1.  Sparse pairs (planned by step s-1) and the decisions run
    // on the main stream A, the decisions after C's consecutive pairs.
    hipStream_t Cs = e->stream_c;
    HIPCK(hipStreamWaitEvent(Cs, e->ev_b[slot_s], 0), "wait");
    if (e->step_no >= 2) HIPCK(hipStreamWaitEvent(Cs, e->pub_ev[(e->step_no - 2) % kSnap], 0), "wait");
    // persistent motion-search grids, autotuned on the consecutive launch
    int64_t sparse_max = 0;
    for (const HostStream& s : e->streams) if (s.open && !s.done) sparse_max += s.sparse_tiles_max;
    int bucket = 0;
    while (bucket < 31 && (int64_t(1) << (bucket + 1)) <= consec_tiles) ++bucket;
    const bool flow = e->params.search == 2;
    TuneCand wgs{e->me_fixed, e->me_fixed};
    if (!e->me_fixed && !flow) {
        if (e->tune_win && e->tune_win->bucket != bucket) {   // the bucket changed: drop the window
            e->tune_win->bucket = -1;
            e->tune_win = nullptr;
        }
        int cand;
        if (e->tune_win) {
            cand = e->tune_win->cand;
        } else {
            cand = me_candidate(e, bucket);
            // windows start once the pipeline is full
            if (e->tune[bucket].best < 0 && consec_tiles > 0 && e->step_no >= kTuneStart) {
                vsa_engine::TunePending* tp = &e->tune_ring[e->tune_head];
                e->tune_head = (e->tune_head + 1) % kTuneRing;
                if (tp->bucket >= 0) tune_harvest(e, *tp, true);   // the slot's previous window
                tp->bucket = bucket;
                tp->cand = cand;
                HIPCK(hipEventRecord(tp->ev0, A), "event");      // A holds only earlier steps' work here
                e->tune_win = tp;
                e->tune_left = kTuneWindow;
            }
        }
        wgs = kTuneCands[cand];
    }
    const int me_cap = std::min(e->has8 ? me_max_wgs_per_cu(8) : 64, e->has10 ? me_max_wgs_per_cu(10) : 64);
    auto me_grid = [&](int64_t tiles, int w) {
        w = std::max(1, std::min(w, me_cap));
        int g = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)w * e->cus);
        if (g >= 8) g -= g % 8;   // whole groups of one workgroup per XCD
        return g;
    };
    const int grid_c = me_grid(consec_tiles, wgs.consec), grid_s = me_grid(sparse_max, wgs.sparse);
    // coarse-to-fine frame pairs: their own kernel, within its occupancy
    const bool hier = e->params.search == 1;
    const int mh_cap = std::min(e->has8 ? me_hier_max_wgs_per_cu(8) : 64, e->has10 ? me_hier_max_wgs_per_cu(10) : 64);
    auto mh_grid = [&](int64_t tiles, int w) {
        w = std::max(1, std::min(w, mh_cap));
        int g = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)w * e->cus);
        if (g >= 8) g -= g % 8;
        return g;
    };
    // its waves spend most of their time waiting for their tile's loads, so its
    // grids take every workgroup a CU holds
    const int grid_hc = hier ? mh_grid(consec_tiles, mh_cap) : 0;
    const int grid_hs = hier ? mh_grid(sparse_max, mh_cap) : 0;
    // consecutive partials alternate by step parity; sparse task lists, jobs
    // and maps too (read the previous step's, write the next)
    TilePartial* cpart = e->d_partials + (size_t)par * e->partials_cap;
    TilePartial* spart = e->d_partials + (size_t)2 * e->partials_cap;
    const size_t sp_cap = (size_t)M * kMaxTasksPerStream;
    PairTask* sparse_prev = e->d_sparse + (size_t)(par ^ 1) * sp_cap;
    PairTask* sparse_next = e->d_sparse + (size_t)par * sp_cap;
    TileJob* sjobs_prev = e->d_sjobs + (size_t)(par ^ 1) * sp_cap;
    TileJob* sjobs_next = e->d_sjobs + (size_t)par * sp_cap;
    int32_t* smap_prev = e->d_smap + (size_t)(par ^ 1) * e->partials_cap;
    int32_t* smap_next = e->d_smap + (size_t)par * e->partials_cap;
    if (flow && (consec_tiles > 0 || sparse_max > 0) && (!e->d_flow_c || !e->d_flow_s))
        return fail(VSA_E_STATE, "dense flow scratch missing");
    // one launch per sample width that an open stream has
    if (flow) {
        if (consec_tiles > 0)
            HIPCK(launch_flow_list(e->d_sds, cjobs, M, cmap, consec_tiles, nullptr, 0, false, e->d_flow_c,
                                   e->flow_unit, cpart, consec_tiles, e->cus, Cs),
                  "dense flow launch");
    } else if (consec_tiles > 0 && !hier) {
        if (e->has8)
            HIPCK(launch_me(8, e->d_sds, cjobs, M, cmap, consec_tiles, nullptr, 0, false, cpart, nullptr, nullptr,
                            grid_c, Cs, timing(1, true, true)), "motion search launch");
        if (e->has10)
            HIPCK(launch_me(10, e->d_sds, cjobs, M, cmap, consec_tiles, nullptr, 0, false, cpart, nullptr, nullptr,
                            grid_c, Cs, timing(2, true, true)), "motion search launch");
    } else if (consec_tiles > 0) {
        // every consecutive pair is a frame pair: the coarse-to-fine kernel alone
        if (e->has8)
            HIPCK(launch_me_hier(8, e->d_sds, cjobs, M, cmap, consec_tiles, nullptr, 0, cpart, nullptr, nullptr,
                                 grid_hc, Cs, timing(1, true, true)), "motion search launch");
        if (e->has10)
            HIPCK(launch_me_hier(10, e->d_sds, cjobs, M, cmap, consec_tiles, nullptr, 0, cpart, nullptr, nullptr,
                                 grid_hc, Cs, timing(2, true, true)), "motion search launch");
    }
    if (hier && e->step_no >= 1) {
        // the planned deep-check pairs (frame pairs, coarse-to-fine) on this
        // stream, once the previous step's decisions that planned them are
        // done, beside the field pairs' full search on the main stream.  The
        // decisions of this step wait for ev_c, so the planning counter and
        // the job list they read are not reused before they have run.
        HIPCK(hipStreamWaitEvent(Cs, e->pub_ev[(e->step_no - 1) % kSnap], 0), "wait");
        if (e->has8 || !e->has10)
            HIPCK(launch_me_hier(8, e->d_sds, sjobs_prev, (int32_t)sp_cap, smap_prev, 0, e->d_cur, par ^ 1, spart,
                                 nullptr, nullptr, grid_hs, Cs), "motion search launch");
        if (e->has10)
            HIPCK(launch_me_hier(10, e->d_sds, sjobs_prev, (int32_t)sp_cap, smap_prev, 0, e->d_cur, par ^ 1, spart,
                                 nullptr, nullptr, grid_hs, Cs), "motion search launch");
    }
    HIPCK(hipEventRecord(e->ev_c[slot_s], Cs), "event");
    // the first sparse launch also clears the counter this step's decisions
    // plan into: the 8-bit one runs unless only 10-bit streams are open
    const bool sparse8 = e->has8 || !e->has10;
    if (flow)
        HIPCK(launch_flow_list(e->d_sds, sjobs_prev, (int32_t)sp_cap, smap_prev, 0, e->d_cur, par ^ 1, true,
                               e->d_flow_s, e->flow_unit, spart, std::max<int64_t>(sparse_max, 1), e->cus, A),
              "dense flow launch");
    // (with the coarse-to-fine search these are the field pairs' launches; the
    // deep-check pairs went to the search stream above)
    if (sparse8 && !flow)
        HIPCK(launch_me(8, e->d_sds, sjobs_prev, (int32_t)sp_cap, smap_prev, 0, e->d_cur, par ^ 1, true, spart,
                        nullptr, nullptr, grid_s, A, timing(3, true, !e->has10)), "motion search launch");
    if (e->has10 && !flow)
        HIPCK(launch_me(10, e->d_sds, sjobs_prev, (int32_t)sp_cap, smap_prev, 0, e->d_cur, par ^ 1, !sparse8, spart,
                        nullptr, nullptr, grid_s, A, timing(3, !sparse8, true)), "motion search launch");
    HIPCK(hipStreamWaitEvent(A, e->ev_c[slot_s], 0), "wait");
    if (!e->no_intensity) HIPCK(hipStreamWaitEvent(A, e->ev_h[slot_s], 0), "wait");
    const int sn = (int)(e->step_no % kSnap);
    HIPCK(launch_finish_decide(e->d_sds, e->d_states, d_steps, n_steps, e->dp, cpart, spart,
                               sparse_prev, sparse_next, e->d_cur, e->d_out_frames, kFramesCap, e->d_out_shots,
                               kShotsCap, e->d_log, kLogCapPerStream, e->d_closed, par, e->d_snap + sn,
                               sjobs_next, smap_next, A, n_steps > 0 ? timing(4, true, true) : LaunchTiming{}),
          "decide launch");
    prof(5, 1, A);
    // the decision kernel wrote this step's cursors into h_snap[sn]; vsa_collect
    // reads them once pub_ev[sn] has completed
    HIPCK(hipEventRecord(e->pub_ev[sn], A), "event");
    HIPCK(hipEventRecord(e->ev_a[slot_s], A), "event");
    if (e->tune_win && --e->tune_left == 0) {
        HIPCK(hipEventRecord(e->tune_win->ev1, A), "event");
        e->tune_win = nullptr;
    }
    e->prof_step += 1;
    e->step_no += 1;
    if (user) HIPCK(hipStreamWaitEvent(user, e->ev_a[slot_s], 0), "wait");
    for (HostStream& s : e->streams)
        if (s.open && s.pending) { s.pending = false; s.next_frame += 1; }
    e->pushed_since_drain += step_push;
    e->pushed_total += step_push;
    e->pushed_cum[sn] = e->pushed_total;
    const uint64_t t_end = now_ns();
    e->counters[10] += t_built - t_start;
    e->counters[11] += t_upload - t_built;
    e->counters[12] += t_end - t_upload;
    e->counters[13] += t_end - t_start;
    e->counters[0] += 1;
    e->counters[7] += (uint64_t)n_consec;
    for (int i = 0; i < n_consec; ++i) e->counters[8] += (uint64_t)(consec[i].tiles >= 0 ? e->streams[consec[i].sid].sd.B_L : 0);
    return VSA_OK;
}

vsa_status vsa_sync(vsa_engine* e) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    return drain(e);
}

vsa_status vsa_collect(vsa_engine* e, int64_t* steps_published) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    vsa_status st = collect(e);
    if (steps_published) *steps_published = e->pub_step + 1;
    return st;
}

int32_t vsa_poll_frames_all(vsa_engine* e, int32_t* sids, vsa_frame_result* out, int32_t cap) {
    if (!e || ((!out || !sids) && cap > 0) || cap < 0) return fail(VSA_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lk(e->mu);
    int32_t n = 0;
    for (int sid = 0; sid < e->max_streams && n < cap; ++sid) {
        HostStream& s = e->streams[sid];
        if (!s.open) continue;
        while (n < cap && !s.fq.empty()) {
            sids[n] = sid;
            out[n++] = s.fq.front();
            s.fq.pop_front();
        }
    }
    return n;
}

int32_t vsa_poll_frames(vsa_engine* e, int32_t sid, vsa_frame_result* out, int32_t cap) {
    if (!e || (!out && cap > 0) || cap < 0) return fail(VSA_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    int32_t n = 0;
    while (n < cap && !s->fq.empty()) { out[n++] = s->fq.front(); s->fq.pop_front(); }
    return n;
}

int32_t vsa_poll_shots(vsa_engine* e, int32_t sid, vsa_shot_result* out, int32_t cap) {
    if (!e || (!out && cap > 0) || cap < 0) return fail(VSA_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    int32_t n = 0;
    while (n < cap && !s->sq.empty()) { out[n++] = s->sq.front(); s->sq.pop_front(); }
    return n;
}

vsa_status vsa_get_motion(vsa_engine* e, int32_t sid, int64_t frame, int8_t* mv, int32_t cap_blocks,
                          int32_t* nbx, int32_t* nby) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    const int bx = s->sd.wl[0] / 8, by = s->sd.hl[0] / 8;
    if (nbx) *nbx = bx;
    if (nby) *nby = by;
    if (!mv) return VSA_OK;
    if (s->sd.search == 2) return fail(VSA_E_UNSUPPORTED, "the dense flow (search 2) keeps no block motion field");
    if (cap_blocks < bx * by) return fail(VSA_E_INVAL, "output too small");
    // pair (frame -> frame+1) exists once frame+1 has been stepped and is still in the ring
    if (frame < 0 || frame + 1 >= s->next_frame || frame < s->next_frame - s->sd.rs)
        return fail(VSA_E_INVAL, "frame not held on the device");
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    HIPCK(hipStreamSynchronize(e->stream_b), "sync");
    HIPCK(hipStreamSynchronize(e->stream_c), "sync");
    HIPCK(hipStreamSynchronize(e->stream), "sync");
    HIPCK(hipMemcpy(mv, s->sd.mv + (frame % s->sd.rs) * s->sd.B_L * 2, (size_t)s->sd.B_L * 2,
                    hipMemcpyDeviceToHost), "motion copy");
    return VSA_OK;
}

vsa_status vsa_get_histogram(vsa_engine* e, int32_t sid, int64_t frame, uint32_t* bins, int32_t cap,
                             int32_t* nbins) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    const int nb = 1 << s->sd.bits;
    if (nbins) *nbins = nb;
    if (!s->sd.tileh) return fail(VSA_E_STATE, "the engine was created with no_intensity");
    if (!bins) return VSA_OK;
    if (cap < nb) return fail(VSA_E_INVAL, "output too small");
    if (frame < 0 || frame >= s->next_frame || frame < s->next_frame - s->sd.rs)
        return fail(VSA_E_INVAL, "frame not held on the device");
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    HIPCK(hipStreamSynchronize(e->stream_b), "sync");
    HIPCK(hipStreamSynchronize(e->stream_c), "sync");
    HIPCK(hipStreamSynchronize(e->stream), "sync");
    HIPCK(hipMemcpy(bins, s->sd.ring + (frame % s->sd.rs) * s->sd.slot_bytes + s->sd.offH,
                    sizeof(uint32_t) * nb, hipMemcpyDeviceToHost), "histogram copy");
    return VSA_OK;
}

vsa_status vsa_stream_close(vsa_engine* e, int32_t sid) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    // records of this stream still in flight carry its epoch and are dropped
    // when published; queued steps still read its memory, so the memory is
    // only reused once the main stream has passed them
    free_stream(e, sid);
    bool any8 = false, any10 = false;
    for (const HostStream& o : e->streams) {
        if (o.open && o.sd.bits == 10) any10 = true;
        if (o.open && o.sd.bits == 8) any8 = true;
    }
    e->has8 = any8;
    e->has10 = any10;
    return VSA_OK;
}

vsa_status vsa_engine_counters(vsa_engine* e, uint64_t* out, int32_t n) {
    if (!e || !out || n < 0) return fail(VSA_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(e->mu);
    int open = 0;
    for (const HostStream& s : e->streams) if (s.open) ++open;
    e->counters[1] = (uint64_t)open;
    e->counters[4] = e->used;
    e->counters[5] = e->budget;
    for (int32_t i = 0; i < n && i < 14; ++i) out[i] = e->counters[i];
    return VSA_OK;
}

int32_t vsa_engine_tuning(vsa_engine* e, int32_t bucket, int32_t* best, int32_t* wgs, int32_t* windows,
                          double* step_ms, int32_t cap) {
    if (!e || bucket < 0 || bucket >= 32 || cap < 0) return fail(VSA_E_INVAL, "bad argument");
    if (cap > 0 && (!best || !wgs || !windows || !step_ms)) return fail(VSA_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(e->mu);
    const auto& b = e->tune[bucket];
    if (best) *best = b.best;
    for (int c = 0; c < kTuneN && c < cap; ++c) {
        wgs[2 * c] = kTuneCands[c].consec;
        wgs[2 * c + 1] = kTuneCands[c].sparse;
        windows[c] = b.n[c];
        step_ms[c] = b.n[c] ? b.ms[c] / kTuneWindow : 0.0;
    }
    return kTuneN;
}

int32_t vsa_debug_measure_log(vsa_engine* e, int32_t sid, int32_t* keys, int32_t cap) {
    if (!e) return fail(VSA_E_INVAL, "NULL engine");
    std::lock_guard<std::mutex> lk(e->mu);
    HostStream* s = get_stream(e, sid);
    if (!s) return fail(VSA_E_INVAL, "no such stream");
    if (!e->d_log) return fail(VSA_E_STATE, "engine created without debug_log");
    HIPCK(hipSetDevice(e->device), "hipSetDevice");
    HIPCK(hipStreamSynchronize(e->stream_b), "sync");
    HIPCK(hipStreamSynchronize(e->stream_c), "sync");
    HIPCK(hipStreamSynchronize(e->stream), "sync");
    DecideState st;
    HIPCK(hipMemcpy(&st, e->d_states + sid, sizeof st, hipMemcpyDeviceToHost), "state");
    const int64_t n = std::min<int64_t>(st.log_count, kLogCapPerStream);
    if (keys && cap > 0) {
        const int64_t m = std::min<int64_t>(n, cap);
        HIPCK(hipMemcpy(keys, e->d_log + (int64_t)sid * kLogCapPerStream * 6, sizeof(int32_t) * 6 * m,
                        hipMemcpyDeviceToHost), "log");
    }
    return (int32_t)n;
}

// ---- test hooks -------------------------------------------------------------

vsa_status vsa_debug_levels(const vsa_params* pp, const void* luma, int32_t W, int32_t H, int64_t pitch,
                            int32_t bits, uint16_t* out, int64_t cap, int64_t* n_out) {
    if (!luma || (bits != 8 && bits != 10)) return fail(VSA_E_INVAL, "bad argument");
    vsa_params p;
    if (pp) p = *pp; else vsa_default_params(&p);
    vsa_status st = check_params(p);
    if (st != VSA_OK) return st;
    Geo g;
    st = make_geo(W, H, p, kMaxKmax, g);
    if (st != VSA_OK) return st;
    const int b = bits == 8 ? 1 : 2;
    if (pitch < (int64_t)W * b) return fail(VSA_E_INVAL, "pitch smaller than a row");
    StreamDesc sd;
    layout(g, W, H, bits, kMaxKmax, sd);
    sd.rs = 1;
    int64_t n = 0;
    for (int d = 0; d < sd.nlev; ++d) n += (int64_t)sd.wl[d] * sd.hl[d];
    n += 2 * (int64_t)sd.wf * sd.hf;
    if (n_out) *n_out = n;
    if (!out) return VSA_OK;
    if (cap < n) return fail(VSA_E_INVAL, "output too small");
    uint8_t *ring = nullptr, *plane = nullptr, *dsd = nullptr, *ddesc = nullptr;
    FrameInfo* info = nullptr;
    std::vector<uint8_t> host(sd.slot_bytes);
    hipError_t err = hipMalloc(&ring, sd.slot_bytes);
    if (err == hipSuccess) err = hipMalloc(&plane, pitch * H);
    if (err == hipSuccess) err = hipMalloc(&info, sizeof(FrameInfo));
    if (err == hipSuccess) err = hipMalloc(&dsd, sizeof(StreamDesc));
    if (err == hipSuccess) err = hipMalloc(&ddesc, sizeof(StepStream) + 256);
    if (err == hipSuccess) err = hipMemset(ring, 0, sd.slot_bytes);
    if (err == hipSuccess) err = hipMemcpy(plane, luma, pitch * H, hipMemcpyHostToDevice);
    sd.ring = ring;
    sd.info = info;
    StepStream ss;
    std::memset(&ss, 0, sizeof ss);
    ss.sid = 0; ss.has_frame = 1; ss.frame = 0; ss.ended_T = -1;
    ss.src = plane; ss.src_pitch = pitch;
    ss.k1_tiles = pyramid_tiles(sd);
    ss.k1_prefix = 0;
    int32_t k1idx = 0;
    if (err == hipSuccess) err = hipMemcpy(dsd, &sd, sizeof sd, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(ddesc, &ss, sizeof ss, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(ddesc + 256, &k1idx, sizeof k1idx, hipMemcpyHostToDevice);
    if (err == hipSuccess)
        err = launch_pyramid(bits, sd.L, reinterpret_cast<StreamDesc*>(dsd), reinterpret_cast<StepStream*>(ddesc),
                             reinterpret_cast<int32_t*>(ddesc + 256), 1, ss.k1_tiles, nullptr, nullptr, nullptr);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err == hipSuccess) err = hipMemcpy(host.data(), ring, sd.slot_bytes, hipMemcpyDeviceToHost);
    for (void* q : {(void*)ring, (void*)plane, (void*)info, (void*)dsd, (void*)ddesc}) if (q) (void)hipFree(q);
    if (err != hipSuccess) return hip_fail(err, "debug levels");
    int64_t k = 0;
    auto put = [&](int64_t off, int w, int h, int pitch_s) {
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                const int64_t o = off + ((int64_t)y * pitch_s + x) * b;
                out[k++] = b == 1 ? host[o] : (uint16_t)(host[o] | (host[o + 1] << 8));
            }
    };
    for (int d = 0; d < sd.nlev; ++d) put(sd.off[d], sd.wl[d], sd.hl[d], sd.pl[d]);
    put(sd.offU, sd.wf, sd.hf, sd.pf);
    put(sd.offD, sd.wf, sd.hf, sd.pf);
    return VSA_OK;
}

// The flow kernels address a plane with 24-bit row products and 32-bit byte
// offsets: sides below 2^24 and fewer than 2^31 samples.
static bool flow_plane_fits(int64_t w, int64_t h) { return w < (1 << 24) && h < (1 << 24) && w * h < (1ll << 31); }

int64_t vsa_flow_scratch_bytes(int32_t w, int32_t h) {
    if (w < 8 || h < 8) return fail(VSA_E_INVAL, "plane smaller than one 8 x 8 patch");
    if (!flow_plane_fits(w, h)) return fail(VSA_E_INVAL, "plane of 2^31 samples or more");
    return flow_scratch_bytes(w, h);
}

vsa_status vsa_flow_pair(const vsa_params* pp, const void* I, const void* J, int32_t w, int32_t h, int64_t pitch_bytes,
                         int32_t bits, void* scratch, int64_t scratch_bytes, double* flow, double* results,
                         void* hip_stream) {
    if (!I || !J || !scratch || !results || (bits != 8 && bits != 10)) return fail(VSA_E_INVAL, "bad argument");
    if (w < 8 || h < 8) return fail(VSA_E_INVAL, "plane smaller than one 8 x 8 patch");
    if (!flow_plane_fits(w, h)) return fail(VSA_E_INVAL, "plane of 2^31 samples or more");
    if (pitch_bytes < (int64_t)w * (bits == 8 ? 1 : 2)) return fail(VSA_E_INVAL, "pitch smaller than a row");
    if (bits == 10 && ((pitch_bytes & 1) || (reinterpret_cast<uintptr_t>(I) & 1) || (reinterpret_cast<uintptr_t>(J) & 1)))
        return fail(VSA_E_INVAL, "10-bit planes and pitch must be 2-byte aligned");
    if (scratch_bytes < flow_scratch_bytes(w, h)) return fail(VSA_E_INVAL, "scratch smaller than vsa_flow_scratch_bytes");
    vsa_params p;
    if (pp) p = *pp; else vsa_default_params(&p);
    HIPCK(launch_flow_pair(static_cast<const uint8_t*>(I), static_cast<const uint8_t*>(J), w, h, pitch_bytes, bits,
                           p.a0, p.a_static_fx, static_cast<uint8_t*>(scratch), flow, results,
                           static_cast<hipStream_t>(hip_stream)),
          "flow pair launch");
    return VSA_OK;
}

vsa_status vsa_debug_flow_pair(const vsa_params* pp, const uint16_t* I, const uint16_t* J, int32_t w, int32_t h,
                               int32_t bits, double* flow, double* dbl, int32_t* is_static) {
    if (!I || !J || (bits != 8 && bits != 10) || w < 8 || h < 8) return fail(VSA_E_INVAL, "bad argument");
    if (!flow_plane_fits(w, h)) return fail(VSA_E_INVAL, "plane of 2^31 samples or more");
    const int maxv = bits == 8 ? 255 : 1023;
    for (int64_t i = 0; i < (int64_t)w * h; ++i)
        if (I[i] > maxv || J[i] > maxv) return fail(VSA_E_INVAL, "sample out of range");
    const int64_t n = (int64_t)w * h;
    const int64_t sb = flow_scratch_bytes(w, h);
    uint8_t *dI = nullptr, *dJ = nullptr, *scr = nullptr;
    double *dflow = nullptr, *dres = nullptr;
    hipError_t err = hipMalloc(&dI, 2 * n);
    if (err == hipSuccess) err = hipMalloc(&dJ, 2 * n);
    if (err == hipSuccess) err = hipMalloc(&scr, sb);
    if (err == hipSuccess && flow) err = hipMalloc(&dflow, sizeof(double) * 2 * n);
    if (err == hipSuccess) err = hipMalloc(&dres, sizeof(double) * 5);
    if (err == hipSuccess) err = hipMemcpy(dI, I, 2 * n, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(dJ, J, 2 * n, hipMemcpyHostToDevice);
    vsa_status st = VSA_OK;
    if (err == hipSuccess) {
        // the samples go in as 16-bit words whatever their width
        st = vsa_flow_pair(pp, dI, dJ, w, h, 2 * (int64_t)w, 10, scr, sb, dflow, dres, nullptr);
        if (st == VSA_OK) err = hipDeviceSynchronize();
    }
    double res[5] = {0, 0, 0, 0, 0};
    if (err == hipSuccess && st == VSA_OK) err = hipMemcpy(res, dres, sizeof res, hipMemcpyDeviceToHost);
    if (err == hipSuccess && st == VSA_OK && flow) err = hipMemcpy(flow, dflow, sizeof(double) * 2 * n, hipMemcpyDeviceToHost);
    for (void* q : {(void*)dI, (void*)dJ, (void*)scr, (void*)dflow, (void*)dres})
        if (q) (void)hipFree(q);
    if (st != VSA_OK) return st;
    if (err != hipSuccess) return fail(VSA_E_DEVICE, hipGetErrorString(err));
    if (dbl) { dbl[0] = res[0]; dbl[1] = res[1]; dbl[2] = res[2]; dbl[3] = res[3]; }
    if (is_static) *is_static = res[4] != 0.0 ? 1 : 0;
    return VSA_OK;
}

vsa_status vsa_debug_pair(const vsa_params* pp, const uint16_t* I, const uint16_t* J, int32_t w, int32_t h,
                          int32_t bits, int32_t force_zero_mv, int8_t* mv, int32_t* sad, int64_t* ints,
                          double* dbl) {
    if (!I || !J || (bits != 8 && bits != 10) || w < 8 || h < 8) return fail(VSA_E_INVAL, "bad argument");
    vsa_params p;
    if (pp) p = *pp; else vsa_default_params(&p);
    vsa_status st = check_params(p);
    if (st != VSA_OK) return st;
    if (p.search == 2) return fail(VSA_E_UNSUPPORTED, "the dense flow pair measure is vsa_debug_flow_pair");
    const int b = bits == 8 ? 1 : 2;
    const int maxv = bits == 8 ? 255 : 1023;
    for (int64_t i = 0; i < (int64_t)w * h; ++i)
        if (I[i] > maxv || J[i] > maxv) return fail(VSA_E_INVAL, "sample out of range");
    StreamDesc sd;
    std::memset(&sd, 0, sizeof sd);
    sd.active = 1; sd.W = w; sd.H = h; sd.bits = bits; sd.L = 0; sd.Lcap = 0; sd.Lf = 0; sd.ltop = 0;
    sd.nlev = 1; sd.k_max = 1; sd.rs = 2;
    sd.wl[0] = w; sd.hl[0] = h; sd.pl[0] = (int)round_up(w, 64); sd.off[0] = 0;
    sd.wf = w; sd.hf = h; sd.pf = sd.pl[0]; sd.offU = sd.offD = 0;
    sd.slot_bytes = round_up((int64_t)sd.pl[0] * h * b, 256);
    sd.B_L = (w / 8) * (h / 8);
    sd.search = p.search;
    std::vector<uint8_t> host(2 * sd.slot_bytes, 0);
    for (int s = 0; s < 2; ++s) {
        const uint16_t* src = s == 0 ? I : J;
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                const int64_t o = s * sd.slot_bytes + ((int64_t)y * sd.pl[0] + x) * b;
                host[o] = (uint8_t)(src[(int64_t)y * w + x] & 0xff);
                if (b == 2) host[o + 1] = (uint8_t)(src[(int64_t)y * w + x] >> 8);
            }
    }
    PairTask t;
    std::memset(&t, 0, sizeof t);
    t.sid = 0; t.kind = MK_CONSEC; t.ref = 0; t.oth = 1; t.level = 0; t.result = -1;
    t.tiles = frame_pair_tiles(p.search, w, h); t.tile_prefix = 0;
    t.flags = TF_DEBUG | (force_zero_mv ? TF_ZERO_MV : 0);
    uint8_t *ring = nullptr, *dsd = nullptr, *dt = nullptr, *djob = nullptr;
    int32_t* dmap = nullptr;
    FrameInfo* info = nullptr;
    TilePartial* part = nullptr;
    int8_t* dmv = nullptr;
    int32_t* dsad = nullptr;
    int64_t* dints = nullptr;
    double* ddbl = nullptr;
    const int B = sd.B_L;
    hipError_t err = hipMalloc(&ring, host.size());
    if (err == hipSuccess) err = hipMalloc(&dsd, sizeof sd);
    if (err == hipSuccess) err = hipMalloc(&dt, sizeof t);
    if (err == hipSuccess) err = hipMalloc(&djob, sizeof(TileJob));
    if (err == hipSuccess) err = hipMalloc(&dmap, sizeof(int32_t) * t.tiles);
    if (err == hipSuccess) err = hipMemset(dmap, 0, sizeof(int32_t) * t.tiles);   // every tile: job 0
    if (err == hipSuccess) err = hipMalloc(&info, 2 * sizeof(FrameInfo));
    if (err == hipSuccess) err = hipMalloc(&part, sizeof(TilePartial) * t.tiles);
    if (err == hipSuccess) err = hipMalloc(&dmv, 2 * (size_t)B);
    if (err == hipSuccess) err = hipMalloc(&dsad, sizeof(int32_t) * B);
    if (err == hipSuccess) err = hipMalloc(&dints, sizeof(int64_t) * 9);
    if (err == hipSuccess) err = hipMalloc(&ddbl, sizeof(double) * 4);
    sd.ring = ring;
    sd.info = info;
    if (err == hipSuccess) err = hipMemcpy(ring, host.data(), host.size(), hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(dsd, &sd, sizeof sd, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(dt, &t, sizeof t, hipMemcpyHostToDevice);
    const TileJob job = make_tile_job(sd, t, nullptr);
    if (err == hipSuccess) err = hipMemcpy(djob, &job, sizeof job, hipMemcpyHostToDevice);
    const DecideParams dp = decide_params(p, 0);
    if (err == hipSuccess && !p.search)
        err = launch_me(bits, reinterpret_cast<StreamDesc*>(dsd), reinterpret_cast<TileJob*>(djob), 1, dmap, t.tiles,
                        nullptr, 0, false, part, dmv, dsad, std::min(t.tiles, 1024), nullptr);
    if (err == hipSuccess && p.search)
        err = launch_me_hier(bits, reinterpret_cast<StreamDesc*>(dsd), reinterpret_cast<TileJob*>(djob), 1, dmap,
                             t.tiles, nullptr, 0, part, dmv, dsad, std::min(t.tiles, 1024), nullptr);
    if (err == hipSuccess)
        err = launch_finish(reinterpret_cast<StreamDesc*>(dsd), reinterpret_cast<PairTask*>(dt), 1, t.tiles,
                            nullptr, nullptr, part, nullptr, dp, dints, ddbl, 1, 0, nullptr);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err == hipSuccess && mv) err = hipMemcpy(mv, dmv, 2 * (size_t)B, hipMemcpyDeviceToHost);
    if (err == hipSuccess && sad) err = hipMemcpy(sad, dsad, sizeof(int32_t) * B, hipMemcpyDeviceToHost);
    if (err == hipSuccess && ints) err = hipMemcpy(ints, dints, sizeof(int64_t) * 9, hipMemcpyDeviceToHost);
    if (err == hipSuccess && dbl) err = hipMemcpy(dbl, ddbl, sizeof(double) * 4, hipMemcpyDeviceToHost);
    for (void* q : {(void*)ring, (void*)dsd, (void*)dt, (void*)info, (void*)part, (void*)dmv, (void*)dsad,
                    (void*)dints, (void*)ddbl, (void*)djob, (void*)dmap})
        if (q) (void)hipFree(q);
    if (err != hipSuccess) return hip_fail(err, "debug pair");
    return VSA_OK;
}

vsa_status vsa_debug_finish(const int64_t* ints, int64_t n, double a0, double* out) {
    if (!ints || !out || n < 0) return fail(VSA_E_INVAL, "bad argument");
    if (n == 0) return VSA_OK;
    for (int64_t i = 0; i < n; ++i)
        if (ints[8 * i + 5] <= 0 || ints[8 * i + 7] <= 0) return fail(VSA_E_INVAL, "N and B must be positive");
    int64_t* di = nullptr;
    double* dd = nullptr;
    hipError_t err = hipMalloc(&di, sizeof(int64_t) * 8 * n);
    if (err == hipSuccess) err = hipMalloc(&dd, sizeof(double) * 4 * n);
    if (err == hipSuccess) err = hipMemcpy(di, ints, sizeof(int64_t) * 8 * n, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = launch_finish_debug(di, n, a0, dd, nullptr);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err == hipSuccess) err = hipMemcpy(out, dd, sizeof(double) * 4 * n, hipMemcpyDeviceToHost);
    if (di) (void)hipFree(di);
    if (dd) (void)hipFree(dd);
    if (err != hipSuccess) return hip_fail(err, "debug finish");
    return VSA_OK;
}

vsa_status vsa_debug_decide(const vsa_params* pp, int32_t k_max, int32_t dense, int32_t T, const double* act,
                            const double* swr, const uint8_t* stat, const double* v, const double* F,
                            const double* S, const double* P, vsa_frame_result* recs, vsa_shot_result* shots,
                            int32_t shots_cap, int32_t* n_shots, int32_t* keys, int32_t keys_cap,
                            int32_t* n_keys) {
    if (T < 1 || !act || !swr || !stat || !v || !F || !S || !P || !recs || (!shots && shots_cap > 0))
        return fail(VSA_E_INVAL, "bad argument");
    vsa_params p;
    if (pp) p = *pp; else vsa_default_params(&p);
    vsa_status st = check_params(p);
    if (st != VSA_OK) return st;
    const int kmax = k_max ? k_max : p.k_max;
    if (kmax < 1 || kmax > kMaxKmax) return fail(VSA_E_INVAL, "k_max must be in 1..15");
    StreamDesc sd;
    std::memset(&sd, 0, sizeof sd);
    sd.active = 1; sd.k_max = kmax; sd.rs = 2 * kmax + 4 + kAhead; sd.L = 0; sd.Lcap = kMaxLevels - 1;
    sd.ltop = kMaxLevels - 1; sd.nlev = kMaxLevels; sd.Lf = 0;
    for (int d = 0; d < kMaxLevels; ++d) { sd.wl[d] = 16; sd.hl[d] = 16; }
    sd.wf = 16; sd.hf = 16;
    const int kw = kmax + 2;
    const size_t nT = (size_t)T;
    DecideState ds;
    init_state(ds);
    const DecideParams dp = decide_params(p, dense);
    uint8_t* mem = nullptr;
    size_t off[16];
    size_t sz = 0;
    auto reserve = [&](int i, size_t bytes) { off[i] = sz; sz += round_up(bytes, 256); };
    reserve(0, sizeof(FrameInfo) * sd.rs);
    reserve(1, sizeof(DecideState));
    reserve(2, sizeof(PairResult) * kResSlots);
    reserve(3, sizeof(double) * nT);
    reserve(4, sizeof(double) * nT);
    reserve(5, nT);
    reserve(6, sizeof(double) * 3 * nT);
    reserve(7, sizeof(double) * kw * nT);
    reserve(8, sizeof(double) * kw * nT);
    reserve(9, sizeof(double) * kw * nT);
    reserve(10, sizeof(vsa_frame_result) * nT);
    reserve(11, sizeof(vsa_shot_result) * std::max(shots_cap, 1));
    reserve(12, sizeof(int32_t) * 2);
    const int log_cap = std::max(keys_cap, 0);
    reserve(13, sizeof(int32_t) * 6 * std::max(log_cap, 1));
    hipError_t err = hipMalloc(&mem, sz);
    if (err != hipSuccess) return hip_fail(err, "debug decide");
    auto at = [&](int i) { return mem + off[i]; };
    sd.info = reinterpret_cast<FrameInfo*>(at(0));
    err = hipMemset(mem, 0, sz);
    if (err == hipSuccess) err = hipMemcpy(at(1), &ds, sizeof ds, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(3), act, sizeof(double) * nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(4), swr, sizeof(double) * nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(5), stat, nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(6), v, sizeof(double) * 3 * nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(7), F, sizeof(double) * kw * nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(8), S, sizeof(double) * kw * nT, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(at(9), P, sizeof(double) * kw * nT, hipMemcpyHostToDevice);
    int32_t counts[2] = {0, 0};
    if (err == hipSuccess)
        err = launch_decide_replay(sd, reinterpret_cast<DecideState*>(at(1)), reinterpret_cast<PairResult*>(at(2)),
                                   dp, T, reinterpret_cast<double*>(at(3)), reinterpret_cast<double*>(at(4)),
                                   reinterpret_cast<uint8_t*>(at(5)), reinterpret_cast<double*>(at(6)),
                                   reinterpret_cast<double*>(at(7)), reinterpret_cast<double*>(at(8)),
                                   reinterpret_cast<double*>(at(9)), reinterpret_cast<vsa_frame_result*>(at(10)),
                                   reinterpret_cast<vsa_shot_result*>(at(11)), shots_cap,
                                   reinterpret_cast<int32_t*>(at(12)), keys ? reinterpret_cast<int32_t*>(at(13)) : nullptr,
                                   log_cap, reinterpret_cast<int32_t*>(at(12)) + 1, nullptr);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err == hipSuccess) err = hipMemcpy(recs, at(10), sizeof(vsa_frame_result) * nT, hipMemcpyDeviceToHost);
    if (err == hipSuccess) err = hipMemcpy(counts, at(12), sizeof counts, hipMemcpyDeviceToHost);
    if (err == hipSuccess && shots && shots_cap > 0)
        err = hipMemcpy(shots, at(11), sizeof(vsa_shot_result) * std::min(counts[0], shots_cap), hipMemcpyDeviceToHost);
    if (err == hipSuccess && keys && log_cap > 0)
        err = hipMemcpy(keys, at(13), sizeof(int32_t) * 6 * std::min(counts[1], log_cap), hipMemcpyDeviceToHost);
    (void)hipFree(mem);
    if (err != hipSuccess) return hip_fail(err, "debug decide");
    if (n_shots) *n_shots = counts[0];
    if (n_keys) *n_keys = counts[1];
    return VSA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Offline form: one whole clip with temporal look-ahead batching.
//
// The streaming engine advances each stream by one frame per step, so a lone
// stream pays a step's launches and host work for every frame.  Here all
// frames of the clip are at hand and are taken `chunk` at a time (the first
// chunk shorter, so that the decisions start early):
//   ingest stream (P), per chunk:
//     K1  pyramid, fields and intensity measure of every frame of the chunk
//         (one launch);
//     K2  motion search of every consecutive pair that ends in the chunk
//         (one persistent launch);
//   decision stream (D), per chunk, once P has finished it:
//     the pairs' finishing arithmetic into the frame records (k_finish);
//     K6, the sequential pass over the new frames until it asks for sparse
//     measures, then rounds of (K2 over the requested pairs, K6) until it
//     waits for frames of the next chunk or, at the end of the clip, has
//     closed the last shot.
// P ingests chunk c+1 while D runs the rounds of chunk c.  The finishing
// arithmetic stays on D: it writes the record of the chunk's first pair,
// whose reference frame is the previous chunk's last, which that chunk's
// decisions may still be labelling.  Each frame of a chunk is a pyramid entry
// of its own: the chunk's stream descriptors are copies of the clip's,
// sharing its ring, motion fields and frame records, each with its own tile
// histograms.  Descriptors, jobs, tile maps, partials and tile histograms are
// double-buffered by chunk parity.  The ring holds two chunks plus the deep
// check's look-back and look-ahead, so an ingested chunk never overwrites a
// frame that the pass can still read.  The host learns whether another round
// is needed from the cursor snapshot each decision launch writes into mapped
// memory: it enqueues as many rounds as the previous chunk took before it
// first waits, then four at a time.  K6 runs as k_finish_decide<true>, which
// also computes the fields of later frames ahead of the pass (speculative
// field measures, cached per ring slot), so that an analysis window costs a
// few rounds rather than one per analysed frame.
struct vsa_clip {
    std::mutex mu;
    int device = 0;
    DecideParams dp{};
    bool no_intensity = false;
    int C = 0;                     // frames per chunk
    StreamDesc sd{};               // the clip's descriptor (ring of 2 chunk + 2 k_max + 8 slots)
    int pyr_tiles = 0;             // pyramid tiles per frame
    int pair_tiles = 0;            // motion-search tiles of a consecutive pair
    int sparse_tiles = 0;          // most tiles one round's sparse pairs can have
    int grid_c = 0, grid_s = 0;    // persistent motion-search grids
    int grid_hc = 0, grid_hs = 0;  // and those of the coarse-to-fine kernel (search = 1)
    int cus = 0;                   // compute units (the dense flow's phase grids, search = 2)
    int64_t flow_unit = 0;         // dense flow scratch bytes per tile
    uint8_t* d_flow_c = nullptr;   // C x pair_tiles units (the consecutive pairs of a chunk)
    uint8_t* d_flow_s = nullptr;   // sparse_tiles units
    hipStream_t s = nullptr;       // decisions (D)
    hipStream_t sp = nullptr;      // ingest (P)
    hipEvent_t ev_p[2] = {};       // P has finished the chunk of that parity
    uint8_t* mem = nullptr;        // ring, frame records, motion fields, tile histograms
    StreamDesc* d_sds = nullptr;   // 2 x C descriptors (entry q C + i: frame i of a chunk of parity q)
    DecideState* d_state = nullptr;
    DeviceCursors* d_cur = nullptr;
    vsa_shot_result* d_closed = nullptr;
    uint8_t* d_desc = nullptr;     // per parity: StepStream[C + 2], pyramid list[C], consecutive tasks[C]
    uint8_t* h_desc = nullptr;     // its pinned source (per parity)
    size_t desc_bytes = 0, off_k1 = 0, off_cons = 0;
    DecideState* h_init = nullptr; // pinned source of the decision state's reset
    TileJob* d_cjobs = nullptr;    // 2 x C
    int32_t* d_cmap = nullptr;     // 2 x C x pair_tiles
    TilePartial* d_part = nullptr; // 2 x C x pair_tiles (consecutive), then sparse_tiles
    PairTask* d_sparse = nullptr;  // 2 x kMaxTasksPerStream (by decision-launch parity)
    TileJob* d_sjobs = nullptr;    // 2 x kMaxTasksPerStream
    int32_t* d_smap = nullptr;     // 2 x sparse_tiles
    OutFrame* h_out_frames = nullptr;
    OutFrame* d_out_frames = nullptr;
    OutShot* h_out_shots = nullptr;
    OutShot* d_out_shots = nullptr;
    uint64_t out_cap = 0;
    PubSnap* h_snap = nullptr;     // [2], by decision-launch parity
    PubSnap* d_snap = nullptr;
    double* d_spec = nullptr;      // speculative field cache: rs x (v0, v1, v2, frame)
    uint8_t* d_stage = nullptr;    // host-sourced frames of two chunks
    int64_t stage_pitch = 0, stage_bytes = 0;
    int64_t dec_no = 0;            // decision launches in the current run
    int est_rounds = 8;            // rounds enqueued before the first wait of a chunk
    uint64_t counters[6] = {0};    // chunks, decision launches, host waits, sparse tasks, speculative
                                   // field tasks among them, measures requested by the pass
    int32_t* d_log = nullptr;      // with debug_log: the measures the pass requested (6 int32 each)
    int64_t log_cap = 0, log_n = 0;  // capacity, and the count of the last run
};

namespace {

int64_t clip_info_offset(const StreamDesc& sd) { return sd.slot_bytes * sd.rs; }
int64_t clip_mv_offset(const StreamDesc& sd) {
    return clip_info_offset(sd) + round_up((int64_t)sizeof(FrameInfo) * sd.rs, 256);
}
int64_t clip_tileh_offset(const StreamDesc& sd) { return clip_mv_offset(sd) + round_up((int64_t)sd.rs * sd.B_L * 2, 256); }

// Everything the sequential pass and the sparse pairs of one decision launch
// need: the sparse K2 over the tasks the previous launch planned (it also
// clears the counter this launch plans into), then K6 for the clip's entry.
vsa_status clip_decide(vsa_clip* c, const StepStream* d_entry) {
    const int par = (int)(c->dec_no & 1);
    const size_t tc = kMaxTasksPerStream;
    PairTask* sp_prev = c->d_sparse + (size_t)(par ^ 1) * tc;
    PairTask* sp_next = c->d_sparse + (size_t)par * tc;
    TileJob* sj_prev = c->d_sjobs + (size_t)(par ^ 1) * tc;
    TileJob* sj_next = c->d_sjobs + (size_t)par * tc;
    int32_t* sm_prev = c->d_smap + (size_t)(par ^ 1) * c->sparse_tiles;
    int32_t* sm_next = c->d_smap + (size_t)par * c->sparse_tiles;
    TilePartial* spart = c->d_part + (size_t)2 * c->C * c->pair_tiles;
    if (c->sd.search == 2)
        HIPCK(launch_flow_list(c->d_sds, sj_prev, (int32_t)tc, sm_prev, 0, c->d_cur, par ^ 1, true, c->d_flow_s,
                               c->flow_unit, spart, c->sparse_tiles, c->cus, c->s),
              "dense flow launch");
    else
        HIPCK(launch_me(c->sd.bits, c->d_sds, sj_prev, (int32_t)tc, sm_prev, 0, c->d_cur, par ^ 1, true, spart,
                        nullptr, nullptr, c->grid_s, c->s),
              "motion search launch");
    if (c->sd.search == 1)   // the deep-check pairs among them (frame pairs) take the coarse-to-fine kernel
        HIPCK(launch_me_hier(c->sd.bits, c->d_sds, sj_prev, (int32_t)tc, sm_prev, 0, c->d_cur, par ^ 1, spart,
                             nullptr, nullptr, c->grid_hs, c->s),
              "motion search launch");
    HIPCK(launch_finish_decide(c->d_sds, c->d_state, d_entry, 1, c->dp, c->d_part, spart, sp_prev, sp_next, c->d_cur,
                               c->d_out_frames, c->out_cap, c->d_out_shots, c->out_cap, c->d_log, c->log_cap, c->d_closed, par,
                               c->d_snap + par, sj_next, sm_next, c->s),
          "decide launch");
    c->dec_no += 1;
    c->counters[1] += 1;
    return VSA_OK;
}

// Whether the last decision launch planned sparse tasks (after a wait).
bool clip_pending(const vsa_clip* c) {
    const int64_t j = c->dec_no - 1;
    const uint64_t now = c->h_snap[j & 1].sparse_run;
    const uint64_t before = j >= 1 ? c->h_snap[(j - 1) & 1].sparse_run : 0;
    return now != before;
}

// Where the frames of one run come from.
struct ClipSource {
    const uint8_t* base;
    int64_t stride, pitch;
    int32_t T, src;
};

// Chunks of a clip: the first takes min(C, max(16, C / 4)) frames, so that
// the decisions start before a whole chunk has been ingested; the others C.
int clip_head(int C) { return std::min(C, std::max(16, C / 4)); }
int clip_chunk_start(int C, int ch) { return ch == 0 ? 0 : clip_head(C) + (ch - 1) * C; }
int clip_chunks(int C, int T) { return T <= clip_head(C) ? 1 : 1 + (T - clip_head(C) + C - 1) / C; }

// Fill the descriptors of chunk ch (parity ch & 1) and enqueue its ingest on
// P: host-sourced planes, descriptor upload, K1 (+ intensity), consecutive
// K2; then record ev_p of its parity.  *n_cons receives its consecutive pairs.
vsa_status clip_ingest(vsa_clip* c, const ClipSource& in, int ch, int* n_cons_out, int* ctiles_out) {
    const StreamDesc& sd = c->sd;
    const int C = c->C, q = ch & 1;
    const int f0 = clip_chunk_start(C, ch), n = std::min(ch == 0 ? clip_head(C) : C, in.T - f0);
    const bool last = f0 + n == in.T;
    const int64_t row = (int64_t)sd.W * (sd.bits == 8 ? 1 : 2);
    uint8_t* h = c->h_desc + (size_t)q * c->desc_bytes;
    uint8_t* dd = c->d_desc + (size_t)q * c->desc_bytes;
    StepStream* steps = reinterpret_cast<StepStream*>(h);
    int32_t* k1 = reinterpret_cast<int32_t*>(h + c->off_k1);
    PairTask* cons = reinterpret_cast<PairTask*>(h + c->off_cons);
    uint8_t* stage = c->d_stage ? c->d_stage + (int64_t)q * C * c->stage_bytes : nullptr;
    if (in.src == VSA_SRC_HOST)
        for (int i = 0; i < n; ++i)
            HIPCK(hipMemcpy2DAsync(stage + (int64_t)i * c->stage_bytes, c->stage_pitch,
                                   in.base + (int64_t)(f0 + i) * in.stride, in.pitch, row, sd.H,
                                   hipMemcpyHostToDevice, c->sp),
                  "plane upload");
    int n_cons = 0, ctiles = 0;
    for (int i = 0; i < n; ++i) {
        StepStream& ss = steps[i];
        std::memset(&ss, 0, sizeof ss);
        ss.sid = q * C + i;
        ss.has_frame = 1;
        ss.frame = f0 + i;
        ss.ended_T = -1;
        ss.pts = f0 + i;
        if (in.src == VSA_SRC_HOST) {
            ss.src = stage + (int64_t)i * c->stage_bytes;
            ss.src_pitch = c->stage_pitch;
        } else {
            ss.src = in.base + (int64_t)(f0 + i) * in.stride;
            ss.src_pitch = in.pitch;
        }
        ss.k1_tiles = c->pyr_tiles;
        ss.k1_prefix = i * c->pyr_tiles;
        k1[i] = i;
        if (f0 + i >= 1) {
            PairTask& t = cons[n_cons++];
            std::memset(&t, 0, sizeof t);
            t.sid = q * C + i;
            t.kind = MK_CONSEC;
            t.ref = f0 + i - 1;
            t.oth = f0 + i;
            t.ref_field = t.oth_field = PL_FRAME;
            t.level = sd.L;
            t.result = -1;
            t.tiles = c->pair_tiles;
            t.tile_prefix = ctiles;
            t.flags = TF_MV_RING;
            t.epoch = sd.epoch;
            ss.consec_tiles = c->pair_tiles;
            ss.consec_prefix = ctiles;
            ctiles += c->pair_tiles;
        }
    }
    // the decision entries: the chunk's arrival, then the rounds after it
    for (int k = 0; k < 2; ++k) {
        StepStream& ss = steps[C + k];
        std::memset(&ss, 0, sizeof ss);
        ss.sid = 0;
        ss.has_frame = k == 0;
        ss.frame = k == 0 ? f0 + n - 1 : -1;
        ss.ended_T = last ? in.T : -1;
    }
    HIPCK(hipMemcpyAsync(dd, h, c->desc_bytes, hipMemcpyHostToDevice, c->sp), "descriptor upload");
    const StepStream* d_steps = reinterpret_cast<const StepStream*>(dd);
    const int32_t* d_k1 = reinterpret_cast<const int32_t*>(dd + c->off_k1);
    TileJob* cjobs = c->d_cjobs + (size_t)q * C;
    int32_t* cmap = c->d_cmap + (size_t)q * C * c->pair_tiles;
    TilePartial* cpart = c->d_part + (size_t)q * C * c->pair_tiles;
    HIPCK(launch_pyramid(sd.bits, sd.L, c->d_sds, d_steps, d_k1, n, n * c->pyr_tiles, cjobs, cmap, c->sp),
          "pyramid launch");
    if (!c->no_intensity) HIPCK(launch_intensity(c->d_sds, d_steps, d_k1, n, c->sp), "intensity launch");
    if (ctiles > 0 && sd.search == 2) {
        HIPCK(launch_flow_list(c->d_sds, cjobs, C, cmap, ctiles, nullptr, 0, false, c->d_flow_c, c->flow_unit, cpart,
                               ctiles, c->cus, c->sp),
              "dense flow launch");
    } else if (ctiles > 0) {
        int gc = std::min(sd.search ? c->grid_hc : c->grid_c, ctiles);
        if (gc >= 8) gc -= gc % 8;
        if (sd.search)
            HIPCK(launch_me_hier(sd.bits, c->d_sds, cjobs, C, cmap, ctiles, nullptr, 0, cpart, nullptr, nullptr, gc,
                                 c->sp),
                  "motion search launch");
        else
            HIPCK(launch_me(sd.bits, c->d_sds, cjobs, C, cmap, ctiles, nullptr, 0, false, cpart, nullptr, nullptr, gc,
                            c->sp),
                  "motion search launch");
    }
    HIPCK(hipEventRecord(c->ev_p[q], c->sp), "event");
    *n_cons_out = n_cons;
    *ctiles_out = ctiles;
    return VSA_OK;
}

}  // namespace

extern "C" {

void vsa_clip_destroy(vsa_clip* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->sp) (void)hipStreamSynchronize(c->sp);
    if (c->s) (void)hipStreamSynchronize(c->s);
    void* dev[] = {c->mem, c->d_sds, c->d_state, c->d_cur, c->d_closed, c->d_desc, c->d_cjobs, c->d_cmap,
                   c->d_part, c->d_sparse, c->d_sjobs, c->d_smap, c->d_stage, c->d_spec, c->d_log,
                   c->d_flow_c, c->d_flow_s};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {c->h_desc, c->h_init, c->h_out_frames, c->h_out_shots, c->h_snap};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    for (hipEvent_t ev : c->ev_p)
        if (ev) (void)hipEventDestroy(ev);
    if (c->sp) (void)hipStreamDestroy(c->sp);
    if (c->s) (void)hipStreamDestroy(c->s);
    delete c;
}

vsa_status vsa_clip_create(const vsa_clip_config* cfg, vsa_clip** out) {
    if (!cfg || !out) return fail(VSA_E_INVAL, "NULL argument");
    *out = nullptr;
    vsa_params p;
    if (cfg->params) p = *cfg->params;
    else vsa_default_params(&p);
    vsa_status st = check_params(p);
    if (st != VSA_OK) return st;
    if (cfg->bit_depth != 8 && cfg->bit_depth != 10) return fail(VSA_E_INVAL, "bit_depth must be 8 or 10");
    const int kmax = cfg->k_max ? cfg->k_max : p.k_max;
    if (kmax < 1 || kmax > kMaxKmax) return fail(VSA_E_INVAL, "k_max must be in 1..15");
    if (cfg->schedule != VSA_SCHEDULE_SPARSE && cfg->schedule != VSA_SCHEDULE_DENSE)
        return fail(VSA_E_INVAL, "unknown schedule");
    const int C = cfg->chunk ? cfg->chunk : 256;
    if (C < 1 || C > 4096) return fail(VSA_E_INVAL, "chunk must be in 1..4096");
    if (cfg->me_wgs_per_cu < 0 || cfg->me_wgs_per_cu > 8) return fail(VSA_E_INVAL, "me_wgs_per_cu must be in 0..8");
    Geo g;
    st = make_geo(cfg->width, cfg->height, p, kmax, g);
    if (st != VSA_OK) return st;
    StreamDesc sd;
    layout(g, cfg->width, cfg->height, cfg->bit_depth, kmax, sd);
    sd.search = p.search;
    if (sd.search == 2 && (int64_t)cfg->width * cfg->height >= (1ll << 31))
        return fail(VSA_E_UNSUPPORTED, "frames of 2^31 samples or more with the dense flow");
    st = check_exact_sums(sd);
    if (st != VSA_OK) return st;
    // the chunk being decided, the chunk being ingested beside it, the deep
    // check's look-back (k_max + 1) and look-ahead (k_max + 1), and slack
    sd.rs = 2 * C + 2 * kmax + 8;
    sd.epoch = 1;
    HIPCK(hipSetDevice(cfg->device), "hipSetDevice");
    vsa_clip* c = new vsa_clip;
    std::unique_ptr<vsa_clip, void (*)(vsa_clip*)> guard(c, vsa_clip_destroy);
    c->device = cfg->device;
    c->dp = decide_params(p, cfg->schedule == VSA_SCHEDULE_DENSE);
    c->no_intensity = cfg->no_intensity != 0;
    c->C = C;
    c->pyr_tiles = pyramid_tiles(sd);
    c->pair_tiles = frame_pair_tiles(sd.search, sd.wl[0], sd.hl[0]);
    // one round's sparse pairs: a deep check, or the fields of an analysed
    // frame and of up to kMaxSpec frames after it
    c->sparse_tiles = std::max(max_sparse_tiles(sd), 3 * (1 + kMaxSpec) * field_pair_tiles(sd.search, sd.wf, sd.hf));
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
    const int me_cap = me_max_wgs_per_cu(sd.bits);
    auto grid = [&](int64_t tiles, int w) {
        w = std::max(1, std::min(w, me_cap));
        int gsz = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)w * cus);
        if (gsz >= 8) gsz -= gsz % 8;   // whole groups of one workgroup per XCD
        return gsz;
    };
    c->grid_c = grid((int64_t)C * c->pair_tiles, cfg->me_wgs_per_cu ? cfg->me_wgs_per_cu : 2);
    c->grid_s = grid(c->sparse_tiles, cfg->me_wgs_per_cu ? cfg->me_wgs_per_cu : 4);
    if (sd.search == 2) {
        c->cus = cus;
        c->flow_unit = flow_unit(sd);
    } else if (sd.search) {
        const int mh_cap = me_hier_max_wgs_per_cu(sd.bits);
        auto hgrid = [&](int64_t tiles, int w) {
            w = std::max(1, std::min(w, mh_cap));
            int gsz = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)w * cus);
            if (gsz >= 8) gsz -= gsz % 8;
            return gsz;
        };
        c->grid_hc = hgrid((int64_t)C * c->pair_tiles, cfg->me_wgs_per_cu ? cfg->me_wgs_per_cu : mh_cap);
        c->grid_hs = hgrid(c->sparse_tiles, cfg->me_wgs_per_cu ? cfg->me_wgs_per_cu : mh_cap);
    }
    HIPCK(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking), "hipStreamCreate");
    HIPCK(hipStreamCreateWithFlags(&c->sp, hipStreamNonBlocking), "hipStreamCreate");
    for (hipEvent_t& ev : c->ev_p) HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    const int64_t thb = tile_hist_bytes(sd, !c->no_intensity);
    const int64_t mem_bytes = clip_tileh_offset(sd) + thb * 2 * C;
    auto dalloc = [](void** p_, size_t n) { return hipMalloc(p_, std::max<size_t>(n, 256)) == hipSuccess; };
    c->desc_bytes = round_up(sizeof(StepStream) * (C + 2), 256);
    c->off_k1 = c->desc_bytes;
    c->desc_bytes += round_up(sizeof(int32_t) * C, 256);
    c->off_cons = c->desc_bytes;
    c->desc_bytes += round_up(sizeof(PairTask) * C, 256);
    const size_t tc = kMaxTasksPerStream;
    const size_t cpt = (size_t)C * c->pair_tiles;
    bool ok = dalloc((void**)&c->mem, mem_bytes) && dalloc((void**)&c->d_sds, sizeof(StreamDesc) * 2 * C) &&
              dalloc((void**)&c->d_state, sizeof(DecideState)) && dalloc((void**)&c->d_cur, sizeof(DeviceCursors)) &&
              dalloc((void**)&c->d_closed, sizeof(vsa_shot_result) * kMaxClosed) &&
              dalloc((void**)&c->d_desc, 2 * c->desc_bytes) && dalloc((void**)&c->d_cjobs, sizeof(TileJob) * 2 * C) &&
              dalloc((void**)&c->d_cmap, sizeof(int32_t) * 2 * cpt) &&
              dalloc((void**)&c->d_part, sizeof(TilePartial) * (2 * cpt + c->sparse_tiles)) &&
              dalloc((void**)&c->d_sparse, 2 * sizeof(PairTask) * tc) &&
              dalloc((void**)&c->d_sjobs, 2 * sizeof(TileJob) * tc) &&
              dalloc((void**)&c->d_smap, 2 * sizeof(int32_t) * c->sparse_tiles) &&
              dalloc((void**)&c->d_spec, sizeof(double) * 4 * sd.rs);
    if (ok && sd.search == 2)
        ok = dalloc((void**)&c->d_flow_c, (size_t)(c->flow_unit * (int64_t)cpt)) &&
             dalloc((void**)&c->d_flow_s, (size_t)(c->flow_unit * (int64_t)c->sparse_tiles));
    if (ok && cfg->debug_log) {
        c->log_cap = kLogCapPerStream;
        ok = dalloc((void**)&c->d_log, sizeof(int32_t) * 6 * (size_t)c->log_cap);
    }
    if (!ok) return fail(VSA_E_NOMEM, "clip device buffers");
    // speculative field measures: the sparse schedule only (the dense one
    // computes every frame's fields anyway)
    if (cfg->schedule == VSA_SCHEDULE_SPARSE) c->dp.spec = c->d_spec;
    // records out: a chunk emits at most its frames plus the backlog the pass
    // held (< rs); shots never outnumber frames + 3
    c->out_cap = (uint64_t)(2 * (C + sd.rs) + 64);
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    ok = hipHostMalloc((void**)&c->h_desc, 2 * c->desc_bytes, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&c->h_init, sizeof(DecideState), hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&c->h_out_frames, sizeof(OutFrame) * c->out_cap, mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->d_out_frames, c->h_out_frames, 0) == hipSuccess &&
         hipHostMalloc((void**)&c->h_out_shots, sizeof(OutShot) * c->out_cap, mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->d_out_shots, c->h_out_shots, 0) == hipSuccess &&
         hipHostMalloc((void**)&c->h_snap, 2 * sizeof(PubSnap), mapped) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->d_snap, c->h_snap, 0) == hipSuccess;
    if (!ok) return fail(VSA_E_NOMEM, "clip pinned buffers");
    sd.ring = c->mem;
    sd.info = reinterpret_cast<FrameInfo*>(c->mem + clip_info_offset(sd));
    sd.mv = reinterpret_cast<int8_t*>(c->mem + clip_mv_offset(sd));
    std::vector<StreamDesc> sds(2 * C, sd);
    for (int i = 0; i < 2 * C; ++i)
        sds[i].tileh = c->no_intensity ? nullptr
                                       : reinterpret_cast<uint16_t*>(c->mem + clip_tileh_offset(sd) + thb * i);
    sd.tileh = sds[0].tileh;
    c->sd = sd;
    HIPCK(hipMemcpy(c->d_sds, sds.data(), sizeof(StreamDesc) * 2 * C, hipMemcpyHostToDevice), "descriptor upload");
    *out = guard.release();
    return VSA_OK;
}

// The body of vsa_clip_run, after the argument checks and with the
// analyser's lock held; on failure the caller waits for both streams.
static vsa_status clip_run_body(vsa_clip* c, const void* frames, int64_t frame_stride_bytes, int64_t pitch_bytes,
                                int32_t n_frames, int32_t src, vsa_frame_result* out_frames,
                                vsa_shot_result* out_shots, int32_t shots_cap, int32_t* n_shots) {
    const StreamDesc& sd = c->sd;
    const int64_t row = (int64_t)sd.W * (sd.bits == 8 ? 1 : 2);
    const int C = c->C, T = n_frames;
    if (src == VSA_SRC_HOST && !c->d_stage) {
        c->stage_pitch = round_up(row, 256);
        c->stage_bytes = round_up(c->stage_pitch * sd.H, 256);
        if (hipMalloc((void**)&c->d_stage, (size_t)c->stage_bytes * 2 * C) != hipSuccess) {
            c->d_stage = nullptr;
            return fail(VSA_E_NOMEM, "clip staging");
        }
    }
    // a fresh pass: decision state, cursors, frame records and snapshots
    init_state(*c->h_init);
    HIPCK(hipMemcpyAsync(c->d_state, c->h_init, sizeof(DecideState), hipMemcpyHostToDevice, c->s), "state reset");
    HIPCK(hipMemsetAsync(c->d_cur, 0, sizeof(DeviceCursors), c->s), "cursor reset");
    HIPCK(hipMemsetAsync(sd.info, 0, sizeof(FrameInfo) * sd.rs, c->s), "record reset");
    HIPCK(hipMemsetAsync(c->d_spec, 0xff, sizeof(double) * 4 * sd.rs, c->s), "field cache reset");   // NaN tags
    HIPCK(hipStreamSynchronize(c->s), "reset");
    std::memset(c->h_snap, 0, 2 * sizeof(PubSnap));
    c->dec_no = 0;
    const ClipSource in{static_cast<const uint8_t*>(frames), frame_stride_bytes, pitch_bytes, T, src};
    const int n_chunks = clip_chunks(C, T);
    int n_cons[2] = {0, 0}, ctiles[2] = {0, 0};
    vsa_status st = clip_ingest(c, in, 0, &n_cons[0], &ctiles[0]);
    if (st != VSA_OK) return st;
    uint64_t frames_read = 0, shots_read = 0, run_tasks = 0;
    for (int ch = 0; ch < n_chunks; ++ch) {
        const int q = ch & 1;
        const uint8_t* dd = c->d_desc + (size_t)q * c->desc_bytes;
        const StepStream* d_steps = reinterpret_cast<const StepStream*>(dd);
        // the chunk's pairs into the frame records, then its first decisions
        HIPCK(hipStreamWaitEvent(c->s, c->ev_p[q], 0), "wait");
        if (n_cons[q] > 0)
            HIPCK(launch_finish(c->d_sds, reinterpret_cast<const PairTask*>(dd + c->off_cons), n_cons[q], ctiles[q],
                                nullptr, nullptr, c->d_part + (size_t)q * C * c->pair_tiles, nullptr, c->dp, nullptr,
                                nullptr, (n_cons[q] + 3) / 4, 0, c->s),
                  "finish launch");
        st = clip_decide(c, d_steps + C);
        if (st != VSA_OK) return st;
        // the next chunk's ingest beside this chunk's rounds: the previous
        // chunk's rounds (the last readers of the slots and buffers it
        // reuses) have completed
        if (ch + 1 < n_chunks) {
            st = clip_ingest(c, in, ch + 1, &n_cons[q ^ 1], &ctiles[q ^ 1]);
            if (st != VSA_OK) return st;
        }
        // each round commits at least one iteration of the pass
        const int limit = 4 * (C + sd.rs) + 64;
        int rounds = 0, batch = c->est_rounds;
        for (;;) {
            for (int r = 0; r < batch; ++r, ++rounds) {
                st = clip_decide(c, d_steps + C + 1);
                if (st != VSA_OK) return st;
            }
            HIPCK(hipStreamSynchronize(c->s), "clip chunk");
            c->counters[2] += 1;
            if (!clip_pending(c)) break;
            if (rounds > limit) return fail(VSA_E_DEVICE, "decision pass did not settle");
            batch = 4;
        }
        c->est_rounds = std::min(rounds, 32);
        c->counters[0] += 1;
        // records of this chunk (mapped memory, complete after the wait)
        const PubSnap ps = c->h_snap[(c->dec_no - 1) & 1];
        if (ps.frames_written - frames_read > c->out_cap || ps.shots_written - shots_read > c->out_cap)
            return fail(VSA_E_DEVICE, "clip record ring overflow");
        for (uint64_t i = frames_read; i < ps.frames_written; ++i) {
            const OutFrame& o = c->h_out_frames[i % c->out_cap];
            if (o.r.frame != (int64_t)i || i >= (uint64_t)T) return fail(VSA_E_DEVICE, "clip records out of order");
            out_frames[i] = o.r;
        }
        for (uint64_t i = shots_read; i < ps.shots_written; ++i)
            if (i < (uint64_t)shots_cap) out_shots[i] = c->h_out_shots[i % c->out_cap].r;
        frames_read = ps.frames_written;
        shots_read = ps.shots_written;
        run_tasks = ps.sparse_run;
    }
    HIPCK(hipStreamSynchronize(c->sp), "clip ingest");
    c->counters[3] += run_tasks;
    DecideState fin;
    HIPCK(hipMemcpy(&fin, c->d_state, sizeof fin, hipMemcpyDeviceToHost), "decision state");
    c->counters[4] += (uint64_t)fin.spec_count;
    c->counters[5] += (uint64_t)fin.log_count;
    c->log_n = fin.log_count;
    if (frames_read != (uint64_t)T) return fail(VSA_E_DEVICE, "clip ended with frames missing");
    if (n_shots) *n_shots = (int32_t)shots_read;
    return VSA_OK;
}

vsa_status vsa_clip_run(vsa_clip* c, const void* frames, int64_t frame_stride_bytes, int64_t pitch_bytes,
                        int32_t n_frames, int32_t src, vsa_frame_result* out_frames, vsa_shot_result* out_shots,
                        int32_t shots_cap, int32_t* n_shots) {
    if (!c) return fail(VSA_E_INVAL, "NULL clip");
    if (n_frames < 0) return fail(VSA_E_INVAL, "negative frame count");
    if (n_frames > 0 && (!frames || !out_frames)) return fail(VSA_E_INVAL, "NULL frames or records");
    if (shots_cap < 0 || (shots_cap > 0 && !out_shots)) return fail(VSA_E_INVAL, "bad shot array");
    if (src != VSA_SRC_HOST && src != VSA_SRC_DEVICE_BORROW) return fail(VSA_E_INVAL, "src must be host or device");
    if (n_shots) *n_shots = 0;
    if (n_frames == 0) return VSA_OK;
    std::lock_guard<std::mutex> lk(c->mu);
    const StreamDesc& sd = c->sd;
    const int64_t row = (int64_t)sd.W * (sd.bits == 8 ? 1 : 2);
    if (pitch_bytes < row) return fail(VSA_E_INVAL, "pitch smaller than a row");
    if (n_frames > 1 && frame_stride_bytes < pitch_bytes * (sd.H - 1) + row)
        return fail(VSA_E_INVAL, "frame stride smaller than a frame");
    if (src == VSA_SRC_HOST && sd.bits == 10)
        for (int32_t i = 0; i < n_frames; ++i)
            if (!samples_10bit_ok(static_cast<const uint8_t*>(frames) + (int64_t)i * frame_stride_bytes, pitch_bytes,
                                  sd.W, sd.H))
                return fail(VSA_E_INVAL, "10-bit frame holds a sample above 1023");
    HIPCK(hipSetDevice(c->device), "hipSetDevice");
    const vsa_status st = clip_run_body(c, frames, frame_stride_bytes, pitch_bytes, n_frames, src, out_frames,
                                        out_shots, shots_cap, n_shots);
    if (st != VSA_OK) {
        // nothing queued may still read the caller's frames once the call returns
        (void)hipStreamSynchronize(c->sp);
        (void)hipStreamSynchronize(c->s);
    }
    return st;
}

int32_t vsa_debug_clip_chunks(int32_t chunk, int32_t n_frames, int32_t* starts, int32_t* counts, int32_t cap) {
    const int C = chunk ? chunk : 256;
    if (C < 1 || C > 4096 || n_frames < 0 || cap < 0 || (cap > 0 && (!starts || !counts)))
        return fail(VSA_E_INVAL, "bad argument");
    if (n_frames == 0) return 0;
    const int n = clip_chunks(C, n_frames);
    for (int ch = 0; ch < n && ch < cap; ++ch) {
        starts[ch] = clip_chunk_start(C, ch);
        counts[ch] = std::min(ch == 0 ? clip_head(C) : C, n_frames - starts[ch]);
    }
    return n;
}

vsa_status vsa_clip_counters(vsa_clip* c, uint64_t* out, int32_t n) {
    if (!c || !out || n < 0) return fail(VSA_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lk(c->mu);
    for (int i = 0; i < n && i < 6; ++i) out[i] = c->counters[i];
    return VSA_OK;
}

int32_t vsa_clip_debug_log(vsa_clip* c, int32_t* keys, int32_t cap) {
    if (!c || cap < 0 || (cap > 0 && !keys)) return fail(VSA_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->d_log) return fail(VSA_E_STATE, "clip analyser created without debug_log");
    const int64_t n = std::min(c->log_n, c->log_cap);
    const int64_t k = std::min<int64_t>(n, cap);
    if (k > 0) HIPCK(hipMemcpy(keys, c->d_log, sizeof(int32_t) * 6 * k, hipMemcpyDeviceToHost), "clip log");
    return (int32_t)n;
}

}  // extern "C"
