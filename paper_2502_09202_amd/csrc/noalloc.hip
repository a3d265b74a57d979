// noalloc.hip -- the pair measure of two device planes without any allocation.
//
// vsa_pair_noalloc computes what vsa_debug_pair computes (the motion field,
// exact moments, NCC, SWR, AMM and ACT of one pair, Sec. III.A) with the same
// kernels, for callers that cannot allocate: code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc.  Every intermediate
// (padded copies of the two planes, the stream descriptor, the tile job and
// map, the per-tile partial sums) lives in one file-scope device array,
// `scratch`, of a fixed size; the call only enqueues kernels on the caller's
// stream.  The array's device address is taken once per device with
// hipGetSymbolAddress and passed to the kernels as an argument.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "vsa_internal.h"

namespace vsa {
hipError_t launch_me(int bits, const StreamDesc*, const TileJob*, int32_t, const int32_t*, int32_t,
                     const DeviceCursors*, int32_t, bool, TilePartial*, int8_t*, int32_t*, int, hipStream_t,
                     LaunchTiming);
hipError_t launch_finish(const StreamDesc*, const PairTask*, int32_t, int32_t, const PairTask*, DeviceCursors*,
                         const TilePartial*, PairResult*, const DecideParams&, int64_t*, double*, int, int32_t,
                         hipStream_t);
vsa_status report_error(vsa_status code, const char* msg);
vsa_status report_hip_error(hipError_t e, const char* what);
}  // namespace vsa

using namespace vsa;

namespace {

// Largest plane the array holds: 1024 x 1024 samples of up to 2 bytes (every
// working and field level of the workloads up to 3840 x 2160 fits).
constexpr int kNAMaxW = 1024;
constexpr int kNAMaxH = 1024;
constexpr int kNAMaxTiles = (kNAMaxW / (kBlock * kTBX)) * (kNAMaxH / (kBlock * kTBY));
constexpr int64_t kNAPlane = (int64_t)kNAMaxW * kNAMaxH * 2;
// Layout of the array: plane I, plane J (row pitch rounded up to 64 samples),
// then the small structures, each on its own 256-byte boundary.
constexpr int64_t kOffDesc = 2 * kNAPlane;
constexpr int64_t kOffJob = kOffDesc + 1024;
constexpr int64_t kOffTask = kOffJob + 256;
constexpr int64_t kOffInfo = kOffTask + 256;
constexpr int64_t kOffMap = kOffInfo + 1024;
constexpr int64_t kOffPart = kOffMap + 4 * kNAMaxTiles;
constexpr int64_t kScratchBytes = kOffPart + (int64_t)sizeof(TilePartial) * kNAMaxTiles;
static_assert(sizeof(StreamDesc) <= 1024 && sizeof(TileJob) <= 256 && sizeof(PairTask) <= 256 &&
                  2 * sizeof(FrameInfo) <= 1024,
              "scratch layout");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
vsa_status scratch_ptr(uint8_t** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return report_error(VSA_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return report_hip_error(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_ptr[dev];
    return VSA_OK;
}

// Writes the descriptor, job and task into the array and clears what must
// start at zero: the tile map (every tile belongs to job 0) and the frame
// records.  The partial sums need no clearing: every tile writes its own.
__global__ void k_na_setup(StreamDesc sd, TileJob job, PairTask task, int32_t n_tiles, uint8_t* base) {
    if (threadIdx.x == 0) {
        *reinterpret_cast<StreamDesc*>(base + kOffDesc) = sd;
        *reinterpret_cast<TileJob*>(base + kOffJob) = job;
        *reinterpret_cast<PairTask*>(base + kOffTask) = task;
    }
    int32_t* map = reinterpret_cast<int32_t*>(base + kOffMap);
    for (int i = threadIdx.x; i < n_tiles; i += blockDim.x) map[i] = 0;
    uint32_t* info = reinterpret_cast<uint32_t*>(base + kOffInfo);
    for (int i = threadIdx.x; i < (int)(2 * sizeof(FrameInfo) / 4); i += blockDim.x) info[i] = 0u;
}

// Copies both planes into the array with a row pitch of P samples, the
// columns past the plane's width set to zero (they feed no block).
template <typename T>
__global__ void k_na_copy(const T* __restrict__ I, const T* __restrict__ J, int64_t pitch, int32_t w, int32_t h,
                          int32_t P, int64_t slot, uint8_t* base) {
    const int64_t n = (int64_t)P * h;
    T* dst = reinterpret_cast<T*>(base);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 2 * n; k += (int64_t)gridDim.x * blockDim.x) {
        const int plane = k >= n ? 1 : 0;
        const int64_t r = k - plane * n;
        const int y = (int)(r / P), x = (int)(r % P);
        const T* src = plane ? J : I;
        dst[plane * slot + r] = x < w ? src[(int64_t)y * pitch + x] : (T)0;
    }
}

}  // namespace

extern "C" vsa_status vsa_pair_noalloc(const vsa_params* pp, const void* I, const void* J, int32_t w, int32_t h,
                                       int64_t pitch_bytes, int32_t bits, int32_t force_zero_mv, int8_t* mv,
                                       int64_t* ints, double* dbl, void* hip_stream) {
    if (!I || !J || (bits != 8 && bits != 10)) return report_error(VSA_E_INVAL, "bad argument");
    if (w < 8 || h < 8) return report_error(VSA_E_INVAL, "plane smaller than one 8x8 block");
    if (w > kNAMaxW || h > kNAMaxH)
        return report_error(VSA_E_INVAL, "plane larger than the no-alloc maximum of 1024 x 1024 samples");
    const int b = bits == 8 ? 1 : 2;
    if (pitch_bytes < (int64_t)w * b) return report_error(VSA_E_INVAL, "pitch smaller than a row");
    if (b == 2 && ((pitch_bytes & 1) || (reinterpret_cast<uintptr_t>(I) & 1) || (reinterpret_cast<uintptr_t>(J) & 1)))
        return report_error(VSA_E_INVAL, "10-bit planes and pitch must be 2-byte aligned");
    vsa_params p;
    if (pp) p = *pp; else vsa_default_params(&p);
    if (p.block != 8 || p.radius != 8) return report_error(VSA_E_UNSUPPORTED, "block must be 8 and radius 8");
    if (p.search != 0) return report_error(VSA_E_UNSUPPORTED, "the no-alloc pair measure takes the full search");
    uint8_t* base = nullptr;
    vsa_status st = scratch_ptr(&base);
    if (st != VSA_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);

    // one "stream" of two frames at level 0: slot 0 holds I, slot 1 holds J
    const int P = (w + 63) / 64 * 64;
    StreamDesc sd;
    memset(&sd, 0, sizeof sd);
    sd.active = 1; sd.W = w; sd.H = h; sd.bits = bits; sd.nlev = 1; sd.k_max = 1; sd.rs = 2;
    sd.wl[0] = w; sd.hl[0] = h; sd.pl[0] = P; sd.off[0] = 0;
    sd.wf = w; sd.hf = h; sd.pf = P;
    sd.slot_bytes = ((int64_t)P * h * b + 255) / 256 * 256;
    sd.ring = base;
    sd.info = reinterpret_cast<FrameInfo*>(base + kOffInfo);
    sd.B_L = (w / 8) * (h / 8);
    PairTask t;
    memset(&t, 0, sizeof t);
    t.kind = MK_CONSEC; t.ref = 0; t.oth = 1; t.result = -1;
    t.tiles = me_tiles(w, h);
    t.flags = TF_DEBUG | (force_zero_mv ? TF_ZERO_MV : 0);
    const TileJob job = make_tile_job(sd, t, nullptr);

    hipLaunchKernelGGL(k_na_setup, dim3(1), dim3(256), 0, s, sd, job, t, t.tiles, base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip_error(e, "no-alloc setup");
    const int64_t n = 2 * (int64_t)P * h;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (b == 1)
        hipLaunchKernelGGL(k_na_copy<uint8_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint8_t*>(I),
                           static_cast<const uint8_t*>(J), pitch_bytes, w, h, P, sd.slot_bytes, base);
    else
        hipLaunchKernelGGL(k_na_copy<uint16_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint16_t*>(I),
                           static_cast<const uint16_t*>(J), pitch_bytes / 2, w, h, P, sd.slot_bytes / 2, base);
    e = hipGetLastError();
    if (e != hipSuccess) return report_hip_error(e, "no-alloc plane copy");
    DecideParams dp;
    memset(&dp, 0, sizeof dp);
    dp.a0 = p.a0;
    dp.a_static_fx = p.a_static_fx;
    const StreamDesc* dsd = reinterpret_cast<const StreamDesc*>(base + kOffDesc);
    e = launch_me(bits, dsd, reinterpret_cast<const TileJob*>(base + kOffJob), 1,
                  reinterpret_cast<const int32_t*>(base + kOffMap), t.tiles, nullptr, 0, false,
                  reinterpret_cast<TilePartial*>(base + kOffPart), mv, nullptr, std::min(t.tiles, 1024), s,
                  LaunchTiming{});
    if (e == hipSuccess)
        e = launch_finish(dsd, reinterpret_cast<const PairTask*>(base + kOffTask), 1, t.tiles, nullptr, nullptr,
                          reinterpret_cast<const TilePartial*>(base + kOffPart), nullptr, dp, ints, dbl, 1, 0, s);
    if (e != hipSuccess) return report_hip_error(e, "no-alloc pair");
    return VSA_OK;
}
