// k_flow.hip -- the dense inverse search flow pair measure (search = 2).
//
// The paper's motion field is dense inverse search optical flow (Sec. III.A,
// its reference [8]).  This is that method with fixed work, so that it is
// reproducible to the bit: the pair's planes and up to two box-downscaled
// copies (coarsest first); 8 x 8 patches every 4 samples (plus one flush
// with the right / bottom edge); per patch eight inverse-compositional steps
// u <- u - H^-1 sum g (J(x + u) - T(x)) with H = sum g g^T + 64 I, central-
// difference gradients, J sampled bilinearly with clamped coordinates, each
// component clamped to +-32; the flow at a pixel is the average of the
// covering patches' vectors weighted by 1 / max(1, |J(x + u) - I(x)|).  The
// measures: NCC of I against J warped by the flow, AMM = mean flow length.
//
// Everything is IEEE double with no contraction, every sum in a fixed order:
// a patch's 64 terms (row-major) as a balanced binary tree, which a group of
// 16 lanes forms exactly (four terms of one column per lane: the levels over
// a row's columns by lane permutes, the next two in the lane, the last by a
// row mirror); a longer
// list (a row's pixels, then the rows) in runs of 64 lanes (zeros past the
// end), each run a tree (a wavefront's butterfly), the runs' sums added in
// order.  Sixteen lanes per patch for the search, one lane per pixel for
// densification, one wavefront per run of a row for the measure sums and one
// for the rows.
#include "pair_finish.h"

#include <algorithm>

namespace vsa {

namespace {

constexpr int kFP = 8;            // patch edge
constexpr int kFS = 4;            // patch spacing
constexpr int kFScales = 2;       // coarser scales
constexpr int kFIters = 8;        // inverse-compositional steps per patch and scale
constexpr double kFLambda = 64.0; // added to the Hessian's diagonal
constexpr double kFUmax = 32.0;   // displacement components clamped to +-kFUmax

struct FPlane {
    const uint16_t* px;
    int w, h;
};

// A plane has fewer than 2^31 samples and sides below 2^24 (the entries
// refuse larger ones), so a 24-bit row product and a 32-bit byte offset from
// the plane's base reach every sample.
__device__ __forceinline__ int fat(const FPlane& P, int x, int y) {
    const uint32_t off = 2u * (__umul24((uint32_t)y, (uint32_t)P.w) + (uint32_t)x);
    return (int)*reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(P.px) + off);
}

__device__ __forceinline__ double fbilin(const FPlane& J, double X, double Y) {
    const double xc = fmin(fmax(X, 0.0), (double)(J.w - 1));
    const double yc = fmin(fmax(Y, 0.0), (double)(J.h - 1));
    const int x0 = (int)floor(xc), y0 = (int)floor(yc);
    const int x1 = min(x0 + 1, J.w - 1), y1 = min(y0 + 1, J.h - 1);
    const double fx = xc - x0, fy = yc - y0;
    const double a = fat(J, x0, y0), b = fat(J, x1, y0), c = fat(J, x0, y1), d = fat(J, x1, y1);
    const double top = a + fx * (b - a);
    const double bot = c + fx * (d - c);
    return top + fy * (bot - top);
}

// Patch origins along an axis of n samples: k * kFS while the patch fits,
// then one flush with the edge if the grid stops short of it.
__device__ __host__ __forceinline__ int forigins(int n) {
    if (n < kFP) return 0;
    const int k = (n - kFP) / kFS + 1;
    return k + (((k - 1) * kFS + kFP < n) ? 1 : 0);
}
__device__ __forceinline__ int forigin(int n, int i) {
    const int k = (n - kFP) / kFS + 1;
    return i < k ? i * kFS : n - kFP;
}

// Samples of either width into a dense uint16 plane.
__global__ void k_flow_load(const uint8_t* src, int64_t pitch_bytes, int w, int h, int bits, uint16_t* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)w * h) return;
    const int y = (int)(i / w), x = (int)(i - (int64_t)y * w);
    const uint8_t* row = src + (int64_t)y * pitch_bytes;
    dst[i] = bits == 8 ? (uint16_t)row[x] : reinterpret_cast<const uint16_t*>(row)[x];
}

// One 2 x 2 box step, rounding half up; a trailing odd row or column dropped.
__global__ void k_flow_down(const uint16_t* src, int w, int h, uint16_t* dst) {
    const int dw = w / 2, dh = h / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)dw * dh) return;
    const int y = (int)(i / dw), x = (int)(i - (int64_t)y * dw);
    const uint16_t* r0 = src + (int64_t)(2 * y) * w + 2 * x;
    const uint16_t* r1 = r0 + w;
    dst[i] = (uint16_t)(((int)r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
}

// Sum over the 8 lanes of a half-row (lane-xor 1, 2, 4; the halves of the
// 16-lane DPP rows), in every lane of it: lane-xor 1 and 2 by quad permutes;
// after them the four lanes of a quad hold the same sum, so the third level
// takes any lane of the other quad (the half-row mirror).  Each level adds
// the same two values as a balanced tree, in either order.
__device__ __forceinline__ double half_row_tree(double v) {
    v = v + dpp_f64<0xB1>(v);     // quad_perm [1, 0, 3, 2]: lane ^ 1
    v = v + dpp_f64<0x4E>(v);     // quad_perm [2, 3, 0, 1]: lane ^ 2
    v = v + dpp_f64<0x141>(v);    // row_half_mirror: the other quad of the half-row
    return v;
}

// Lanes per patch in the patch search, PL = 8 or 16: each lane holds
// 64 / PL pixels of one column of its patch (rows (64 / PL) (sub >> 3) ..
// + 64 / PL - 1 of column sub & 7), so that the lanes of one load read few
// rows.  Eight lanes (a whole column each) issue fewer instructions per patch
// and suit the pair lists, which have patches to spare; sixteen give a single
// pair twice the groups in flight.
constexpr int kPLList = 8;
constexpr int kPLPair = 16;

// The 64-term balanced tree of a patch (terms in row-major order) held by a
// group of PL lanes (the layout above): levels 1-3 (the columns of a row)
// across the half-row, the next log2(64 / PL) levels (the lane's rows) inside
// the lane, and with 16 lanes the last (the two halves of the patch) across
// the row (the row mirror).  Every lane of the group gets the sum.
template <int PL>
__device__ __forceinline__ double patch_tree(double v[64 / PL]) {
    static_assert(PL == 8 || PL == 16, "a patch group is a half-row or a row of the DPP lanes");
    constexpr int kPR = 64 / PL;
#pragma unroll
    for (int k = 0; k < kPR; ++k) v[k] = half_row_tree(v[k]);
#pragma unroll
    for (int step = 1; step < kPR; step *= 2) {
#pragma unroll
        for (int k = 0; k < kPR; k += 2 * step) v[k] = v[k] + v[k + step];
    }
    if constexpr (PL == 16) return v[0] + dpp_f64<0x140>(v[0]);   // row_mirror: the other half of the row
    return v[0];
}

// The inverse-compositional search of the patch at (px, py) by a group of
// PL lanes holding 64 / PL pixels of one column each (lane `sub`).  (u0, u1)
// start from the coarser scale's dense flow cfx / cfy (cw x ch) at the patch
// centre, or from zero without one.  Every lane of the group returns the
// patch's vector.
template <int PL>
__device__ __forceinline__ void patch_search(const FPlane& I, const FPlane& J, const double* cfx, const double* cfy,
                                             int cw, int ch, int px, int py, int sub, double& ru0, double& ru1) {
    constexpr int kPR = 64 / PL;
    double u0 = 0.0, u1 = 0.0;
    if (cfx) {
        const int cx = min((px + kFP / 2) / 2, cw - 1);
        const int cy = min((py + kFP / 2) / 2, ch - 1);
        u0 = 2.0 * cfx[(int64_t)cy * cw + cx];
        u1 = 2.0 * cfy[(int64_t)cy * cw + cx];
    }
    const int X = px + (sub & 7), Y0 = py + kPR * (sub >> 3);
    // central-difference gradients (exact halves of integer differences)
    double a[kPR], b[kPR], iv[kPR], t[kPR];
#pragma unroll
    for (int k = 0; k < kPR; ++k) {
        const int Y = Y0 + k;
        a[k] = (fat(I, min(X + 1, I.w - 1), Y) - fat(I, max(X - 1, 0), Y)) / 2.0;
        b[k] = (fat(I, X, min(Y + 1, I.h - 1)) - fat(I, X, max(Y - 1, 0))) / 2.0;
        iv[k] = fat(I, X, Y);
    }
#pragma unroll
    for (int k = 0; k < kPR; ++k) t[k] = a[k] * a[k];
    const double h00 = patch_tree<PL>(t) + kFLambda;
#pragma unroll
    for (int k = 0; k < kPR; ++k) t[k] = a[k] * b[k];
    const double h01 = patch_tree<PL>(t);
#pragma unroll
    for (int k = 0; k < kPR; ++k) t[k] = b[k] * b[k];
    const double h11 = patch_tree<PL>(t) + kFLambda;
    const double det = h00 * h11 - h01 * h01;
    for (int it = 0; it < kFIters; ++it) {
        double e[kPR];
#pragma unroll
        for (int k = 0; k < kPR; ++k) e[k] = fbilin(J, X + u0, Y0 + k + u1) - iv[k];
#pragma unroll
        for (int k = 0; k < kPR; ++k) t[k] = a[k] * e[k];
        const double b0 = patch_tree<PL>(t);
#pragma unroll
        for (int k = 0; k < kPR; ++k) t[k] = b[k] * e[k];
        const double b1 = patch_tree<PL>(t);
        const double d0 = (h11 * b0 - h01 * b1) / det;
        const double d1 = (h00 * b1 - h01 * b0) / det;
        u0 = fmin(fmax(u0 - d0, -kFUmax), kFUmax);
        u1 = fmin(fmax(u1 - d1, -kFUmax), kFUmax);
    }
    ru0 = u0;
    ru1 = u1;
}

// 256 / kPLPair patches per 256-lane workgroup, one group of kPLPair lanes
// each.
// cfx / cfy: the coarser scale's dense flow (cw x ch), null at the coarsest
// scale.
__global__ void __launch_bounds__(256) k_flow_patch(FPlane I, FPlane J, const double* cfx, const double* cfy, int cw,
                                                    int ch, double* ux, double* uy) {
    const int nx = forigins(I.w), ny = forigins(I.h);
    const int p = blockIdx.x * (256 / kPLPair) + threadIdx.x / kPLPair;
    if (p >= nx * ny) return;                     // the whole group
    const int sub = threadIdx.x % kPLPair;
    const int j = p / nx, i = p - (p / nx) * nx;
    double u0, u1;
    patch_search<kPLPair>(I, J, cfx, cfy, cw, ch, forigin(I.w, i), forigin(I.h, j), sub, u0, u1);
    if (sub == 0) {
        ux[p] = u0;
        uy[p] = u1;
    }
}

// Patch indices covering sample X along an axis of n samples, ascending:
// regular patches lo .. hi, then the flush patch (index k) when it exists and
// covers X.
__device__ __forceinline__ void fcover(int n, int X, int& lo, int& hi, bool& flush) {
    const int k = (n - kFP) / kFS + 1;
    lo = X >= kFP ? (X - kFS) / kFS : 0;      // the first i with i kFS + kFP > X
    hi = min(k - 1, X / kFS);                 // the last i with i kFS <= X
    flush = forigins(n) > k && X >= n - kFP;
}

// The flow at pixel (X, Y): the average of the covering patches' vectors
// (ux, uy: nx per row of patches), each weighted by 1 / max(1, |J(X + u) - I(X)|),
// the patches taken row by row, ascending, the flush ones last.
__device__ __forceinline__ void densify_at(const FPlane& I, const FPlane& J, const double* ux, const double* uy, int X,
                                           int Y, double& f0, double& f1) {
    const int nx = forigins(I.w);
    const double iv = fat(I, X, Y);
    int jlo, jhi, ilo, ihi;
    bool jf, iff;
    fcover(I.h, Y, jlo, jhi, jf);
    fcover(I.w, X, ilo, ihi, iff);
    const int kx = (I.w - kFP) / kFS + 1, ky = (I.h - kFP) / kFS + 1;
    double n0 = 0.0, n1 = 0.0, den = 0.0;
    for (int jj = jlo; jj <= jhi + (jf ? 1 : 0); ++jj) {
        const int j = jj <= jhi ? jj : ky;                 // the flush row of patches last
        for (int ii = ilo; ii <= ihi + (iff ? 1 : 0); ++ii) {
            const int i = ii <= ihi ? ii : kx;
            const double u0 = ux[j * nx + i], u1 = uy[j * nx + i];
            const double e = fbilin(J, X + u0, Y + u1) - iv;
            const double wgt = 1.0 / fmax(1.0, fabs(e));
            n0 += wgt * u0;
            n1 += wgt * u1;
            den += wgt;
        }
    }
    f0 = n0 / den;
    f1 = n1 / den;
}

// One lane per pixel: the dense flow of a scale.
__global__ void k_flow_densify(FPlane I, FPlane J, const double* ux, const double* uy, double* fx, double* fy) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)I.w * I.h) return;
    const int Y = (int)(q / I.w), X = (int)(q - (int64_t)Y * I.w);
    densify_at(I, J, ux, uy, X, Y, fx[q], fy[q]);
}

// The six measure terms of pixel (X, Y) under flow (u0, u1): x = I, y = J
// warped bilinearly, x^2, y^2, xy and the flow length.
__device__ __forceinline__ void pixel_terms(const FPlane& I, const FPlane& J, int X, int Y, double u0, double u1,
                                            double v[6]) {
    const double x = fat(I, X, Y);
    const double y = fbilin(J, X + u0, Y + u1);
    v[0] = x; v[1] = y; v[2] = x * x; v[3] = y * y; v[4] = x * y;
    v[5] = sqrt(u0 * u0 + u1 * u1);
}

// One wavefront per row (four per workgroup): the row's six measure sums,
// runs of 64 pixels each a tree, the runs added in order.
__global__ void __launch_bounds__(256) k_flow_rows(FPlane I, FPlane J, const double* fx, const double* fy,
                                                   double* rows) {
    const int Y = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (Y >= I.h) return;                         // the whole wavefront
    const int lane = threadIdx.x & 63;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < I.w; c += 64) {
        const int X = c + lane;
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (X < I.w) {
            const int64_t q = (int64_t)Y * I.w + X;
            pixel_terms(I, J, X, Y, fx[q], fy[q], v);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = acc[k] + wave_tree(v[k]);
    }
    if (lane == 0) {
        double* r = rows + 6 * (int64_t)Y;
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] = acc[k];
    }
}

// One wavefront: the rows' sums, then NCC, SWR, AMM, ACT and the static test.
__global__ void __launch_bounds__(64) k_flow_total(const FlowRow* rows, int w, int h, double a0, int a_static_fx,
                                                   double* out) {
    if (blockIdx.x != 0) return;
    const FlowFinish f = flow_finish(rows, w, h, a0, a_static_fx);
    if ((threadIdx.x & 63) != 0) return;
    out[0] = f.ncc;
    out[1] = f.swr;
    out[2] = f.amm;
    out[3] = f.act;
    out[4] = f.is_static ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Pair lists: the engine's and the clip form's pairs with the dense flow.
//
// A pair of a list is cut into one unit per row of its plane: its tiles (in
// the list's tile map) are its rows, and the slot of tile r receives the six
// measure sums of row r, which the finishing kernels add up.  Its scratch
// starts at tile_prefix * unit bytes of the list's scratch (unit: at least
// flow_pair_bytes / rows of every pair the list can hold).  Each phase is one
// launch over the whole list (a persistent grid walking the tiles); a tile
// does the phase's work for its row, or nothing where the phase has fewer
// rows than the pair.

constexpr int kXcdF = 8;          // accelerator complex dies, one L2 each

// Scratch of one pair of a list: per scale (finest first) its I and J
// samples and patch vectors, and for the coarser scales their dense flow
// (the finest scale's flow is consumed where it is made).  Byte offsets from
// the pair's base, each array on a 256-byte boundary.  flow_scale gives one
// scale's entry (w = 0: the pair has no such scale); its loop over the
// scales is unrolled, so a scale chosen at run time is picked by selects
// rather than read from an indexed array (which would live in scratch).
struct FlowScale {
    int w, h;
    int64_t oI, oJ, oux, ouy, ofx, ofy;
};

__host__ __device__ inline int64_t ftake(int64_t& at, int64_t n) {
    const int64_t o = at;
    at += (n + 255) / 256 * 256;
    return o;
}

__host__ __device__ inline FlowScale flow_scale(int w, int h, int k, int64_t* bytes = nullptr) {
    FlowScale r{0, 0, 0, 0, 0, 0, 0, 0};
    int64_t at = 0;
    int cw = w, ch = h;
#pragma unroll
    for (int s = 0; s <= kFScales; ++s) {
        if (s > 0) {
            cw /= 2;
            ch /= 2;
            if (cw < kFP || ch < kFP) break;
        }
        const int64_t px = (int64_t)cw * ch;
        const int64_t pt = (int64_t)forigins(cw) * forigins(ch);
        FlowScale c;
        c.w = cw;
        c.h = ch;
        c.oI = ftake(at, 2 * px);
        c.oJ = ftake(at, 2 * px);
        c.oux = ftake(at, 8 * pt);
        c.ouy = ftake(at, 8 * pt);
        c.ofx = s > 0 ? ftake(at, 8 * px) : 0;
        c.ofy = s > 0 ? ftake(at, 8 * px) : 0;
        if (s == k) r = c;
    }
    if (bytes) *bytes = at;
    return r;
}

// Sample (x, y) of a job's plane (8 or 10 bits, row pitch in samples); with
// cs = Lf + 1 the lower field on the upper field's rows.
__device__ __forceinline__ int job_sample(const uint8_t* P, int pitch, int bits, int cs, int x, int y) {
    const int64_t o = (int64_t)y * pitch + x, op = (int64_t)(y > 0 ? y - 1 : 0) * pitch + x;
    int a, b = 0;
    if (bits == 8) {
        a = P[o];
        if (cs) b = P[op];
    } else {
        const uint16_t* Q = reinterpret_cast<const uint16_t*>(P);
        a = Q[o];
        if (cs) b = Q[op];
    }
    if (!cs) return a;
    const int m = 1 << cs;
    return ((m - 1) * a + b + (m >> 1)) >> cs;
}

enum : int { FL_LOAD = 0, FL_DOWN = 1, FL_PATCH = 2, FL_DENSE = 3, FL_ROWS = 4 };

// One phase over a pair list.  n_tiles: the list's tiles (consecutive
// pairs), or with cur set the sparse pairs planned by the previous step's
// decisions (their count read from cur->sparse_tt[par_prev]).  k: the scale.
template <int PH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_flow_list(const StreamDesc* __restrict__ sds,
                                                   const TileJob* __restrict__ jobs, int32_t n_jobs,
                                                   const int32_t* __restrict__ map, int32_t n_tiles,
                                                   const DeviceCursors* __restrict__ cur, int32_t par_prev,
                                                   uint8_t* __restrict__ scratch, int64_t unit,
                                                   FlowRow* __restrict__ rows, int k,
                                                   unsigned long long* __restrict__ clear_tt) {
    // the sparse list's first phase clears the counter the step's decisions plan into
    if (clear_tt && blockIdx.x == 0 && threadIdx.x == 0) *clear_tt = 0ull;
    const bool sparse = cur != nullptr;
    if (sparse) __builtin_amdgcn_s_setprio(2);
    const int total = sparse ? tt_tiles(cur->sparse_tt[par_prev].v) : n_tiles;
    // one contiguous slice of the tiles per XCD: a pair's neighbouring rows
    // share lines of its planes in that XCD's L2
    int hi = total, first = blockIdx.x, stride = gridDim.x;
    if (gridDim.x >= kXcdF) {
        const int groups = gridDim.x / kXcdF;     // the host launches a multiple of kXcdF
        const int x = blockIdx.x % kXcdF, j = blockIdx.x / kXcdF;
        if (j >= groups) return;
        const int per = (total + kXcdF - 1) / kXcdF;
        const int lo = x * per;
        hi = min(total, lo + per);
        first = lo + j;
        stride = groups;
    }
    __shared__ double red[4][6];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int tile = first; tile < hi; tile += stride) {
        const int idx = map[tile];
        if (idx < 0 || idx >= n_jobs) continue;   // never expected; keeps reads in bounds
        const TileJob& jb = jobs[idx];
        if (!(jb.flags & TF_FLOW)) continue;
        if (sparse) {
            const StreamDesc& sd = sds[jb.sid];
            if (!sd.active || sd.epoch != jb.epoch) continue;   // stream closed since planning
        }
        const int r = tile - jb.tile_prefix;
        if (r < 0 || r >= jb.h) continue;
        uint8_t* base = scratch + (int64_t)jb.tile_prefix * unit;
        if constexpr (PH == FL_LOAD) {
            const FlowScale S = flow_scale(jb.w, jb.h, 0);
            uint16_t* dI = reinterpret_cast<uint16_t*>(base + S.oI) + (int64_t)r * jb.w;
            uint16_t* dJ = reinterpret_cast<uint16_t*>(base + S.oJ) + (int64_t)r * jb.w;
            for (int x = threadIdx.x; x < jb.w; x += 256) {
                dI[x] = (uint16_t)job_sample(jb.I, jb.pitch, jb.bits, jb.cos_I, x, r);
                dJ[x] = (uint16_t)job_sample(jb.J, jb.pitch, jb.bits, jb.cos_J, x, r);
            }
        } else if constexpr (PH == FL_DOWN) {
            const FlowScale S = flow_scale(jb.w, jb.h, k), F = flow_scale(jb.w, jb.h, k - 1);
            if (k < 1 || S.w == 0 || r >= S.h) continue;
            const int sw = F.w, dw = S.w;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const uint16_t* src = reinterpret_cast<const uint16_t*>(base + (side ? F.oJ : F.oI));
                uint16_t* dst = reinterpret_cast<uint16_t*>(base + (side ? S.oJ : S.oI)) + (int64_t)r * dw;
                for (int x = threadIdx.x; x < dw; x += 256) {
                    const uint16_t* r0 = src + (int64_t)(2 * r) * sw + 2 * x;
                    const uint16_t* r1 = r0 + sw;
                    dst[x] = (uint16_t)(((int)r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
                }
            }
        } else if constexpr (PH == FL_PATCH) {
            const FlowScale S = flow_scale(jb.w, jb.h, k), Q = flow_scale(jb.w, jb.h, k + 1);
            if (S.w == 0 || r >= forigins(S.h)) continue;
            const FPlane PI{reinterpret_cast<const uint16_t*>(base + S.oI), S.w, S.h};
            const FPlane PJ{reinterpret_cast<const uint16_t*>(base + S.oJ), S.w, S.h};
            const bool coarse = Q.w != 0;
            const double* cfx = coarse ? reinterpret_cast<const double*>(base + Q.ofx) : nullptr;
            const double* cfy = coarse ? reinterpret_cast<const double*>(base + Q.ofy) : nullptr;
            const int cw = Q.w, ch = Q.h;
            double* ux = reinterpret_cast<double*>(base + S.oux);
            double* uy = reinterpret_cast<double*>(base + S.ouy);
            const int nx = forigins(S.w);
            const int py = forigin(S.h, r);
            const int grp = threadIdx.x / kPLList, sub = threadIdx.x % kPLList;
            for (int i0 = 0; i0 < nx; i0 += 256 / kPLList) {   // the groups of a wavefront stay together
                const int i = i0 + grp;
                if (i < nx) {
                    double u0, u1;
                    patch_search<kPLList>(PI, PJ, cfx, cfy, cw, ch, forigin(S.w, i), py, sub, u0, u1);
                    if (sub == 0) {
                        ux[(int64_t)r * nx + i] = u0;
                        uy[(int64_t)r * nx + i] = u1;
                    }
                }
            }
        } else if constexpr (PH == FL_DENSE) {
            const FlowScale S = flow_scale(jb.w, jb.h, k);
            if (k < 1 || S.w == 0 || r >= S.h) continue;
            const FPlane PI{reinterpret_cast<const uint16_t*>(base + S.oI), S.w, S.h};
            const FPlane PJ{reinterpret_cast<const uint16_t*>(base + S.oJ), S.w, S.h};
            const double* ux = reinterpret_cast<const double*>(base + S.oux);
            const double* uy = reinterpret_cast<const double*>(base + S.ouy);
            double* fx = reinterpret_cast<double*>(base + S.ofx) + (int64_t)r * S.w;
            double* fy = reinterpret_cast<double*>(base + S.ofy) + (int64_t)r * S.w;
            for (int X = threadIdx.x; X < S.w; X += 256) densify_at(PI, PJ, ux, uy, X, r, fx[X], fy[X]);
        } else {
            // the finest scale: each pixel's flow, its measure terms, the
            // row's sums in runs of 64 pixels (one run per wavefront), the
            // runs added in order
            const FlowScale S = flow_scale(jb.w, jb.h, 0);
            const FPlane PI{reinterpret_cast<const uint16_t*>(base + S.oI), jb.w, jb.h};
            const FPlane PJ{reinterpret_cast<const uint16_t*>(base + S.oJ), jb.w, jb.h};
            const double* ux = reinterpret_cast<const double*>(base + S.oux);
            const double* uy = reinterpret_cast<const double*>(base + S.ouy);
            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int c0 = 0; c0 < jb.w; c0 += 256) {
                const int c = c0 + 64 * wave;
                if (c < jb.w) {
                    const int X = c + lane;
                    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    if (X < jb.w) {
                        double u0, u1;
                        densify_at(PI, PJ, ux, uy, X, r, u0, u1);
                        pixel_terms(PI, PJ, X, r, u0, u1, v);
                    }
#pragma unroll
                    for (int q = 0; q < 6; ++q) v[q] = wave_tree(v[q]);
                    if (lane == 0) {
#pragma unroll
                        for (int q = 0; q < 6; ++q) red[wave][q] = v[q];
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    for (int wv = 0; wv < 4 && c0 + 64 * wv < jb.w; ++wv) {
#pragma unroll
                        for (int q = 0; q < 6; ++q) acc[q] = acc[q] + red[wv][q];
                    }
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) {
#pragma unroll
                for (int q = 0; q < 6; ++q) rows[tile].s[q] = acc[q];
            }
        }
    }
}

inline unsigned fgrid(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// Device bytes the flow pair measure of a w x h pair needs (all scales).
int64_t flow_scratch_bytes(int w, int h) {
    int64_t b = 0;
    int cw = w, ch = h;
    for (int k = 0; k <= kFScales; ++k) {
        if (k > 0) {
            cw /= 2;
            ch /= 2;
            if (cw < kFP || ch < kFP) break;
        }
        const int64_t px = (int64_t)cw * ch;
        const int64_t pt = (int64_t)forigins(cw) * forigins(ch);
        b += 2 * ((px * 2 + 255) / 256 * 256);              // I and J samples
        b += 2 * ((pt * 8 + 255) / 256 * 256);              // patch vectors
        b += 2 * ((px * 8 + 255) / 256 * 256);              // dense flow
    }
    b += ((int64_t)h * 6 * 8 + 255) / 256 * 256 + 256;      // row sums, results
    return b;
}

// The flow pair measure of device planes I, J (w x h samples of `bits`, row
// pitch in bytes) into scratch (flow_scratch_bytes(w, h) bytes); the finest
// flow (w x h x 2 doubles, dx dy interleaved) to flow_out if given, and the
// five results (NCC, SWR, AMM, ACT, static) to res_out (device).
hipError_t launch_flow_pair(const uint8_t* I, const uint8_t* J, int w, int h, int64_t pitch, int bits, double a0,
                            int a_static_fx, uint8_t* scratch, double* flow_out, double* res_out, hipStream_t s) {
    uint8_t* at = scratch;
    auto take = [&](int64_t n) { uint8_t* p = at; at += (n + 255) / 256 * 256; return p; };
    struct Scale { uint16_t *I, *J; double *ux, *uy, *fx, *fy; int w, h; };
    Scale sc[kFScales + 1];
    int ns = 0;
    {
        int cw = w, ch = h;
        for (int k = 0; k <= kFScales; ++k) {
            if (k > 0) {
                cw /= 2;
                ch /= 2;
                if (cw < kFP || ch < kFP) break;
            }
            const int64_t px = (int64_t)cw * ch;
            const int64_t pt = (int64_t)forigins(cw) * forigins(ch);
            Scale& c = sc[ns++];
            c.w = cw; c.h = ch;
            c.I = reinterpret_cast<uint16_t*>(take(px * 2));
            c.J = reinterpret_cast<uint16_t*>(take(px * 2));
            c.ux = reinterpret_cast<double*>(take(pt * 8));
            c.uy = reinterpret_cast<double*>(take(pt * 8));
            c.fx = reinterpret_cast<double*>(take(px * 8));
            c.fy = reinterpret_cast<double*>(take(px * 8));
        }
    }
    double* rows = reinterpret_cast<double*>(take((int64_t)h * 6 * 8));
    const int64_t n0 = (int64_t)w * h;
    hipLaunchKernelGGL(k_flow_load, dim3(fgrid(n0, 256)), dim3(256), 0, s, I, pitch, w, h, bits, sc[0].I);
    hipLaunchKernelGGL(k_flow_load, dim3(fgrid(n0, 256)), dim3(256), 0, s, J, pitch, w, h, bits, sc[0].J);
    for (int k = 1; k < ns; ++k) {
        const int64_t n = (int64_t)sc[k].w * sc[k].h;
        hipLaunchKernelGGL(k_flow_down, dim3(fgrid(n, 256)), dim3(256), 0, s, sc[k - 1].I, sc[k - 1].w, sc[k - 1].h,
                           sc[k].I);
        hipLaunchKernelGGL(k_flow_down, dim3(fgrid(n, 256)), dim3(256), 0, s, sc[k - 1].J, sc[k - 1].w, sc[k - 1].h,
                           sc[k].J);
    }
    for (int k = ns - 1; k >= 0; --k) {
        const Scale& c = sc[k];
        const FPlane PI{c.I, c.w, c.h}, PJ{c.J, c.w, c.h};
        const int64_t np = (int64_t)forigins(c.w) * forigins(c.h);
        const double* cfx = k + 1 < ns ? sc[k + 1].fx : nullptr;
        const double* cfy = k + 1 < ns ? sc[k + 1].fy : nullptr;
        const int cw = k + 1 < ns ? sc[k + 1].w : 0, ch = k + 1 < ns ? sc[k + 1].h : 0;
        hipLaunchKernelGGL(k_flow_patch, dim3(fgrid(np, 256 / kPLPair)), dim3(256), 0, s, PI, PJ, cfx, cfy, cw, ch,
                           c.ux, c.uy);
        hipLaunchKernelGGL(k_flow_densify, dim3(fgrid((int64_t)c.w * c.h, 256)), dim3(256), 0, s, PI, PJ, c.ux, c.uy,
                           c.fx, c.fy);
    }
    const FPlane PI{sc[0].I, w, h}, PJ{sc[0].J, w, h};
    hipLaunchKernelGGL(k_flow_rows, dim3(fgrid(h, 4)), dim3(256), 0, s, PI, PJ, sc[0].fx, sc[0].fy, rows);
    hipLaunchKernelGGL(k_flow_total, dim3(1), dim3(64), 0, s, reinterpret_cast<const FlowRow*>(rows), w, h, a0,
                       a_static_fx, res_out);
    if (flow_out) {
        // interleave dx, dy
        hipError_t e = hipMemcpy2DAsync(flow_out, 2 * sizeof(double), sc[0].fx, sizeof(double), sizeof(double), n0,
                                        hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(flow_out + 1, 2 * sizeof(double), sc[0].fy, sizeof(double), sizeof(double), n0,
                                 hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Scratch bytes of one pair of a pair list with a w x h plane.
int64_t flow_pair_bytes(int w, int h) {
    int64_t b = 0;
    (void)flow_scale(w, h, 0, &b);
    return b;
}

// Workgroups of pair-list phase `ph` one compute unit holds at once.
static int flow_phase_wgs_per_cu(int ph) {
    static int cached[5] = {0, 0, 0, 0, 0};
    if (cached[ph] == 0) {
        const void* fns[] = {reinterpret_cast<const void*>(k_flow_list<FL_LOAD>),
                             reinterpret_cast<const void*>(k_flow_list<FL_DOWN>),
                             reinterpret_cast<const void*>(k_flow_list<FL_PATCH>),
                             reinterpret_cast<const void*>(k_flow_list<FL_DENSE>),
                             reinterpret_cast<const void*>(k_flow_list<FL_ROWS>)};
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fns[ph], 256, 0) != hipSuccess || n < 1) n = 1;
        cached[ph] = n;
    }
    return cached[ph];
}

// Every phase of the dense flow over a pair list (jobs, map as for the
// motion search), in order on stream s: the samples, the coarser scales,
// then coarsest first the patch search and (coarser scales) the dense flow,
// and last the finest scale's row sums into rows (one per tile).  With clear
// set (sparse lists), the first phase clears the counter of the other parity.
// Each phase's persistent grid takes as many workgroups as the compute units
// hold of it (cus of them), at most tiles_bound (the list's largest tile
// count), in whole groups of one workgroup per XCD.
hipError_t launch_flow_list(const StreamDesc* sds, const TileJob* jobs, int32_t n_jobs, const int32_t* map,
                            int32_t n_tiles, const DeviceCursors* cur, int32_t par_prev, bool clear, uint8_t* scratch,
                            int64_t unit, TilePartial* rows, int64_t tiles_bound, int cus, hipStream_t s) {
    if (tiles_bound <= 0) return hipSuccess;
    unsigned long long* clear_tt =
        (cur && clear) ? const_cast<unsigned long long*>(&cur->sparse_tt[par_prev ^ 1].v) : nullptr;
    FlowRow* fr = reinterpret_cast<FlowRow*>(rows);
    auto grid = [&](int ph) {
        int g = (int)std::min<int64_t>(tiles_bound, (int64_t)flow_phase_wgs_per_cu(ph) * std::max(cus, 1));
        if (g >= kXcdF) g -= g % kXcdF;
        return dim3(std::max(g, 1));
    };
    const dim3 b(256);
    hipLaunchKernelGGL(k_flow_list<FL_LOAD>, grid(FL_LOAD), b, 0, s, sds, jobs, n_jobs, map, n_tiles, cur, par_prev,
                       scratch, unit, fr, 0, clear_tt);
    for (int k = 1; k <= kFScales; ++k)
        hipLaunchKernelGGL(k_flow_list<FL_DOWN>, grid(FL_DOWN), b, 0, s, sds, jobs, n_jobs, map, n_tiles, cur,
                           par_prev, scratch, unit, fr, k, nullptr);
    for (int k = kFScales; k >= 0; --k) {
        hipLaunchKernelGGL(k_flow_list<FL_PATCH>, grid(FL_PATCH), b, 0, s, sds, jobs, n_jobs, map, n_tiles, cur,
                           par_prev, scratch, unit, fr, k, nullptr);
        if (k > 0)
            hipLaunchKernelGGL(k_flow_list<FL_DENSE>, grid(FL_DENSE), b, 0, s, sds, jobs, n_jobs, map, n_tiles, cur,
                               par_prev, scratch, unit, fr, k, nullptr);
    }
    hipLaunchKernelGGL(k_flow_list<FL_ROWS>, grid(FL_ROWS), b, 0, s, sds, jobs, n_jobs, map, n_tiles, cur, par_prev,
                       scratch, unit, fr, 0, nullptr);
    return hipGetLastError();
}

}  // namespace vsa
