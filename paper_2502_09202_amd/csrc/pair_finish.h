// pair_finish.h -- the finishing arithmetic of a pair measure (device code).
#pragma once
#include "vsa_internal.h"

namespace vsa {

// NCC, SWR, AMM, ACT from the exact integers (operations in this order, no
// contraction: this file is compiled with -ffp-contract=off).
__device__ __forceinline__ void finish_pair(int64_t sx, int64_t sy, int64_t sxx, int64_t syy, int64_t sxy,
                                         int64_t n, int64_t a, int64_t B, double a0, double out[4]) {
    const int64_t cov = n * sxy - sx * sy;
    const int64_t vx = n * sxx - sx * sx;
    const int64_t vy = n * syy - sy * sy;
    double ncc;
    if (vx == 0 && vy == 0) ncc = 1.0;
    else if (vx == 0 || vy == 0) ncc = 0.0;
    else {
        const double x3 = (double)vx * (double)vy;
        const double x4 = __builtin_sqrt(x3);
        const double c = (double)cov / x4;
        ncc = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    }
    const double swr = 1.0 - ncc;
    const double amm = (double)a / (256.0 * (double)B);
    const double act = __builtin_sqrt((amm + a0) * swr);
    out[0] = ncc; out[1] = swr; out[2] = amm; out[3] = act;
}

// A double from another lane of the same 16-lane row by a DPP move of each
// half (CTRL: the DPP lane pattern).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Balanced binary tree sum of the 64 lanes' values (lane order), in every
// lane: a butterfly that adds lane pairs, then pairs of pairs.  Levels 1-2
// (lane ^ 1, lane ^ 2) by DPP quad permutes; after them the lanes of a quad
// hold equal values, so level 3 takes any lane of the other quad of the
// half-row (the half-row mirror) and, likewise, level 4 any lane of the other
// half of the row (the row mirror); levels 5-6 (lane ^ 16, lane ^ 32) by
// shuffles.  Every level adds the tree's two values, in either order.
__device__ __forceinline__ double wave_tree(double v) {
    v = v + dpp_f64<0xB1>(v);     // quad_perm [1, 0, 3, 2]
    v = v + dpp_f64<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    v = v + dpp_f64<0x141>(v);    // row_half_mirror
    v = v + dpp_f64<0x140>(v);    // row_mirror
    v = v + __shfl_xor(v, 16, 64);
    v = v + __shfl_xor(v, 32, 64);
    return v;
}

// A dense flow pair's per-row sums (one per row of its plane, in the slot of
// the row's tile): sum x, sum y, sum x^2, sum y^2, sum xy over the row's
// pixels (x = I, y = J warped by the flow) and the sum of the flow lengths.
struct FlowRow {
    double s[6];
};
static_assert(sizeof(FlowRow) == sizeof(TilePartial), "a flow row sum takes the slot of a tile partial");

struct FlowFinish {
    double ncc, swr, amm, act;
    bool is_static;
};

// The dense flow pair measure from its h row sums (Sec. III.A with the flow
// in place of the block field): the rows' sums in runs of 64 rows, each run a
// tree, the runs added in order; then NCC of I against the warped J, SWR,
// AMM = mean flow length, ACT, and static if 256 AMM < a_static_fx.  Called
// by a whole wavefront; every lane gets the result.
__device__ __forceinline__ FlowFinish flow_finish(const FlowRow* rows, int w, int h, double a0, int a_static_fx) {
    const int lane = threadIdx.x & 63;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < h; c += 64) {
        const int Y = c + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = acc[k] + wave_tree(Y < h ? rows[Y].s[k] : 0.0);
    }
    const double sx = acc[0], sy = acc[1], sxx = acc[2], syy = acc[3], sxy = acc[4], sm = acc[5];
    const double n = (double)w * h;
    const double cov = n * sxy - sx * sy;
    const double vx = n * sxx - sx * sx;
    const double vy = n * syy - sy * sy;
    double ncc;
    if (vx <= 0.0 && vy <= 0.0) ncc = 1.0;
    else if (vx <= 0.0 || vy <= 0.0) ncc = 0.0;
    else {
        const double c = cov / __builtin_sqrt(vx * vy);
        ncc = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    }
    FlowFinish f;
    f.ncc = ncc;
    f.swr = 1.0 - ncc;
    f.amm = sm / n;
    f.act = __builtin_sqrt((f.amm + a0) * f.swr);
    f.is_static = 256.0 * f.amm < (double)a_static_fx;
    return f;
}

}  // namespace vsa
