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

}  // namespace vsa
