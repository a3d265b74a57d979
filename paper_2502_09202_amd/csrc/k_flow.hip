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
// a patch's 64 terms (row-major) as a balanced binary tree, which is exactly
// what a wavefront's butterfly of xor shuffles forms in every lane; a longer
// list (a row's pixels, then the rows) in runs of 64 lanes (zeros past the
// end), each run a tree, the runs' sums added in order.  One wavefront per
// patch for the search, one lane per pixel for densification, one wavefront
// per row for the measure sums and one for the rows.
#include "vsa_internal.h"

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

__device__ __forceinline__ int fat(const FPlane& P, int x, int y) { return (int)P.px[(int64_t)y * P.w + x]; }

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

// Balanced binary tree sum of the 64 lanes' values (lane order), in every lane.
__device__ __forceinline__ double wave_tree(double v) {
#pragma unroll
    for (int step = 1; step < 64; step *= 2) v = v + __shfl_xor(v, step, 64);
    return v;
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

// One wavefront per patch (four per workgroup), lane y * 8 + x on pixel
// (x, y) of the patch: the inverse-compositional search.  cfx / cfy: the
// coarser scale's dense flow (cw x ch), null at the coarsest scale.
__global__ void __launch_bounds__(256) k_flow_patch(FPlane I, FPlane J, const double* cfx, const double* cfy, int cw,
                                                    int ch, double* ux, double* uy) {
    const int nx = forigins(I.w), ny = forigins(I.h);
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= nx * ny) return;                     // the whole wavefront
    const int lane = threadIdx.x & 63;
    const int j = p / nx, i = p - (p / nx) * nx;
    const int px = forigin(I.w, i), py = forigin(I.h, j);
    double u0 = 0.0, u1 = 0.0;
    if (cfx) {
        const int cx = min((px + kFP / 2) / 2, cw - 1);
        const int cy = min((py + kFP / 2) / 2, ch - 1);
        u0 = 2.0 * cfx[(int64_t)cy * cw + cx];
        u1 = 2.0 * cfy[(int64_t)cy * cw + cx];
    }
    const int X = px + (lane & 7), Y = py + (lane >> 3);
    // central-difference gradients (exact halves of integer differences)
    const double a = (fat(I, min(X + 1, I.w - 1), Y) - fat(I, max(X - 1, 0), Y)) / 2.0;
    const double b = (fat(I, X, min(Y + 1, I.h - 1)) - fat(I, X, max(Y - 1, 0))) / 2.0;
    const double iv = fat(I, X, Y);
    const double h00 = wave_tree(a * a) + kFLambda, h01 = wave_tree(a * b), h11 = wave_tree(b * b) + kFLambda;
    const double det = h00 * h11 - h01 * h01;
    for (int it = 0; it < kFIters; ++it) {
        const double e = fbilin(J, X + u0, Y + u1) - iv;
        const double b0 = wave_tree(a * e), b1 = wave_tree(b * e);
        const double d0 = (h11 * b0 - h01 * b1) / det;
        const double d1 = (h00 * b1 - h01 * b0) / det;
        u0 = fmin(fmax(u0 - d0, -kFUmax), kFUmax);
        u1 = fmin(fmax(u1 - d1, -kFUmax), kFUmax);
    }
    if (lane == 0) {
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

// One lane per pixel: the weighted average of the covering patches' vectors.
__global__ void k_flow_densify(FPlane I, FPlane J, const double* ux, const double* uy, double* fx, double* fy) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)I.w * I.h) return;
    const int Y = (int)(q / I.w), X = (int)(q - (int64_t)Y * I.w);
    const int nx = forigins(I.w), ny = forigins(I.h);
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
    (void)ny;
    fx[q] = n0 / den;
    fy[q] = n1 / den;
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
            const double u0 = fx[q], u1 = fy[q];
            const double x = fat(I, X, Y);
            const double y = fbilin(J, X + u0, Y + u1);
            v[0] = x; v[1] = y; v[2] = x * x; v[3] = y * y; v[4] = x * y;
            v[5] = sqrt(u0 * u0 + u1 * u1);
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

// One wavefront: the rows' sums the same way, then NCC, SWR, AMM, ACT and
// the static test.
__global__ void __launch_bounds__(64) k_flow_total(const double* rows, int w, int h, double a0, int a_static_fx,
                                                   double* out) {
    if (blockIdx.x != 0) return;
    const int lane = threadIdx.x & 63;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < h; c += 64) {
        const int Y = c + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = acc[k] + wave_tree(Y < h ? rows[6 * (int64_t)Y + k] : 0.0);
    }
    if (lane != 0) return;
    const double sx = acc[0], sy = acc[1], sxx = acc[2], syy = acc[3], sxy = acc[4], sm = acc[5];
    const double n = (double)w * h;
    const double cov = n * sxy - sx * sy;
    const double vx = n * sxx - sx * sx;
    const double vy = n * syy - sy * sy;
    double ncc;
    if (vx <= 0.0 && vy <= 0.0) ncc = 1.0;
    else if (vx <= 0.0 || vy <= 0.0) ncc = 0.0;
    else {
        const double c = cov / sqrt(vx * vy);
        ncc = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    }
    const double swr = 1.0 - ncc;
    const double amm = sm / n;
    out[0] = ncc;
    out[1] = swr;
    out[2] = amm;
    out[3] = sqrt((amm + a0) * swr);
    out[4] = 256.0 * amm < (double)a_static_fx ? 1.0 : 0.0;
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
        hipLaunchKernelGGL(k_flow_patch, dim3(fgrid(np, 4)), dim3(256), 0, s, PI, PJ, cfx, cfy, cw, ch, c.ux, c.uy);
        hipLaunchKernelGGL(k_flow_densify, dim3(fgrid((int64_t)c.w * c.h, 256)), dim3(256), 0, s, PI, PJ, c.ux, c.uy,
                           c.fx, c.fy);
    }
    const FPlane PI{sc[0].I, w, h}, PJ{sc[0].J, w, h};
    hipLaunchKernelGGL(k_flow_rows, dim3(fgrid(h, 4)), dim3(256), 0, s, PI, PJ, sc[0].fx, sc[0].fy, rows);
    hipLaunchKernelGGL(k_flow_total, dim3(1), dim3(64), 0, s, rows, w, h, a0, a_static_fx, res_out);
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

}  // namespace vsa
