// orc.cpp -- CPU oracle of the per-frame measure engine.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
// CPU-baseline leg of the benchmark; never by the product path.  Plain scalar
// C++17, single-threaded, no intrinsics, built with -O2 -ffp-contract=off so
// every floating-point expression is evaluated exactly as written.  It shares
// no code, header, table or helper with the GPU library.
//
// What it computes follows Sec. III of the paper (Fassold, arXiv 2502.09202):
//   - measures AMM, SWR, ACT from a motion field and NCC (Sec. III.A);
//   - ACT of consecutive frames always, everything else sparse (Sec. III.A);
//   - measures computed on demand and cached (Sec. III.A, last paragraph);
//   - shot boundaries by fast check + deep check (Sec. III.B);
//   - v0, v1, v2 on upper/lower fields, beta = v1/v2 (Sec. III.C);
//   - dynamic keyframes by accumulated ACT (Sec. III.D).
// Where the paper is silent the readings are the ones recorded in the design
// notes (block SAD full search in place of dense optical flow, the 2x2
// rounding pyramid, the fast/deep-check rules, the sampling vote, ...); each
// one is stated at the place it is used below.
#include "orc.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <vector>

namespace {

struct Plane {
    int w = 0, h = 0;
    std::vector<int32_t> px;
    int32_t at(int x, int y) const { return px[(size_t)y * (size_t)w + (size_t)x]; }
};

// Pyramid geometry.  W_l = floor(W_{l-1}/2).  Working level L is the first
// level no wider than wmax; fields (alternate rows, Sec. III.C) are taken at
// Lf = max(0, L - lf_offset); Lcap is the coarsest level that still holds a
// 2 x 2 grid of blocks (used by the long-range pairs of the deep check).
struct Geometry {
    int W = 0, H = 0, L = -1, Lcap = -1, Lf = 0, wf = 0, hf = 0;
    std::vector<int> wl, hl;
};

bool make_geometry(int W, int H, const orc_params& p, Geometry& g) {
    if (W <= 0 || H <= 0 || p.block != 8 || p.wmax < 16) return false;
    g = Geometry();
    g.W = W; g.H = H;
    for (int w = W, h = H; w > 0 && h > 0; w /= 2, h /= 2) { g.wl.push_back(w); g.hl.push_back(h); }
    const int nl = (int)g.wl.size();
    for (int l = 0; l < nl; ++l) if (g.wl[l] <= p.wmax) { g.L = l; break; }
    if (g.L < 0) return false;
    if (g.wl[g.L] / p.block < 2 || g.hl[g.L] / p.block < 2) return false;
    g.Lcap = g.L;
    for (int l = g.L + 1; l < nl; ++l) {
        if (g.wl[l] / p.block >= 2 && g.hl[l] / p.block >= 2) g.Lcap = l; else break;
    }
    g.Lf = std::max(0, g.L - p.lf_offset);
    g.wf = W; g.hf = H / 2;
    for (int l = 1; l <= g.Lf; ++l) { g.wf /= 2; g.hf /= 2; }
    if (g.wf < p.block || g.hf < p.block) return false;
    return true;
}

// Level used by a deep-check pair at distance K: L + ceil(log2 K), capped.
int ceil_log2(int k) { int c = 0; while ((1 << c) < k) ++c; return c; }
int deep_level(const Geometry& g, int K) { return std::min(g.L + ceil_log2(K), g.Lcap); }

// 2 x 2 box average, rounding half up, applied once per level; a trailing odd
// row or column is dropped.
Plane downscale(const Plane& s) {
    Plane d;
    d.w = s.w / 2; d.h = s.h / 2;
    d.px.assign((size_t)d.w * d.h, 0);
    for (int y = 0; y < d.h; ++y)
        for (int x = 0; x < d.w; ++x) {
            int32_t sum = s.at(2 * x, 2 * y) + s.at(2 * x + 1, 2 * y) +
                          s.at(2 * x, 2 * y + 1) + s.at(2 * x + 1, 2 * y + 1);
            d.px[(size_t)y * d.w + x] = (sum + 2) >> 2;
        }
    return d;
}

bool load_frame(const void* base, int W, int H, int64_t pitch, int bits, Plane& out) {
    out.w = W; out.h = H;
    out.px.assign((size_t)W * H, 0);
    const unsigned char* b = (const unsigned char*)base;
    for (int y = 0; y < H; ++y) {
        const unsigned char* row = b + (size_t)y * (size_t)pitch;
        for (int x = 0; x < W; ++x) {
            int32_t v;
            if (bits == 8) v = row[x];
            else { uint16_t u; std::memcpy(&u, row + 2 * (size_t)x, 2); v = u; if (v > 1023) return false; }
            out.px[(size_t)y * W + x] = v;
        }
    }
    return true;
}

// Upper field = even rows, lower field = odd rows (Sec. III.C; the
// introduction's "half width" is read as half height).
Plane field_of(const Plane& f, int parity) {
    Plane o;
    o.w = f.w; o.h = f.h / 2;
    o.px.resize((size_t)o.w * o.h);
    for (int y = 0; y < o.h; ++y)
        for (int x = 0; x < o.w; ++x) o.px[(size_t)y * o.w + x] = f.at(x, 2 * y + parity);
    return o;
}

// The lower field resampled to the rows of the upper field.  At field level
// Lf both fields have a row pitch of p = 2^(Lf+1) full-resolution rows and
// the lower field's rows sit one full-resolution row below the upper field's,
// so the value at upper-field row y lies 1/p of the way from D[y] to D[y-1]:
// ((p-1) D[y] + D[y-1] + p/2) / p, rounded down, D[-1] read as D[0].  Field
// pairs compare the upper field with this plane: an integer motion field can
// not absorb the sub-row offset between the two fields, which would otherwise
// make v0 of progressive content as large as an inter-frame activity
// (Sec. III.C expects it near zero).
Plane cosite_lower(const Plane& D, int Lf) {
    const int s = Lf + 1, p = 1 << s;
    Plane o;
    o.w = D.w; o.h = D.h;
    o.px.resize(D.px.size());
    for (int y = 0; y < D.h; ++y)
        for (int x = 0; x < D.w; ++x) {
            const int32_t a = D.at(x, y), b = D.at(x, y > 0 ? y - 1 : 0);
            o.px[(size_t)y * o.w + x] = ((p - 1) * a + b + p / 2) >> s;
        }
    return o;
}

struct FrameLevels {
    std::vector<Plane> lv;   // levels L..Lcap
    Plane U, D;              // fields at Lf
    Plane Dc;                // D on the rows of U (what field pairs read)
};

void build_levels(const Plane& full, const Geometry& g, FrameLevels& fl) {
    fl.lv.clear();
    Plane cur = full;
    if (g.L == 0) fl.lv.push_back(cur);
    for (int l = 1; l <= g.Lcap; ++l) {
        cur = downscale(cur);
        if (l >= g.L) fl.lv.push_back(cur);
    }
    fl.U = field_of(full, 0);
    fl.D = field_of(full, 1);
    for (int l = 1; l <= g.Lf; ++l) { fl.U = downscale(fl.U); fl.D = downscale(fl.D); }
    fl.Dc = cosite_lower(fl.D, g.Lf);
}

// Candidate order for ties: by squared length, then dy, then dx.
std::vector<int> candidate_ranks(int R) {
    const int n = 2 * R + 1;
    std::vector<std::tuple<int, int, int>> c;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) c.emplace_back(dx * dx + dy * dy, dy, dx);
    std::sort(c.begin(), c.end());
    std::vector<int> rank((size_t)n * n);
    for (size_t i = 0; i < c.size(); ++i) {
        int dy = std::get<1>(c[i]), dx = std::get<2>(c[i]);
        rank[(size_t)(dy + R) * n + (dx + R)] = (int)i;
    }
    return rank;
}

int64_t isqrt64(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

struct PairOut {
    int nbx = 0, nby = 0;
    std::vector<int8_t> mv;
    std::vector<int32_t> sad;
    int64_t sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0, n = 0, a = 0, B = 0;
    bool is_static = false;
    double ncc = 0, swr = 0, amm = 0, act = 0;
    bool ok = true;
};

// NCC, SWR = 1 - NCC, AMM, ACT from the exact integers.  The covariance terms
// are formed exactly in 64-bit integers; NCC = cov / sqrt(vx * vy) in IEEE
// double with the operations in this order; the zero-variance cases follow the
// reading: both constant -> 1, one constant -> 0; the result is clamped to [-1, 1].
// ACT is the geometric mean of (AMM + a0) and SWR.
bool finish(int64_t sx, int64_t sy, int64_t sxx, int64_t syy, int64_t sxy, int64_t n,
            int64_t a, int64_t B, double a0, double out[4]) {
    if (n <= 0 || B <= 0) return false;
    int64_t t1, t2, cov, vx, vy;
    if (__builtin_mul_overflow(n, sxy, &t1) || __builtin_mul_overflow(sx, sy, &t2) ||
        __builtin_sub_overflow(t1, t2, &cov)) return false;
    if (__builtin_mul_overflow(n, sxx, &t1) || __builtin_mul_overflow(sx, sx, &t2) ||
        __builtin_sub_overflow(t1, t2, &vx)) return false;
    if (__builtin_mul_overflow(n, syy, &t1) || __builtin_mul_overflow(sy, sy, &t2) ||
        __builtin_sub_overflow(t1, t2, &vy)) return false;
    double ncc;
    if (vx == 0 && vy == 0) ncc = 1.0;
    else if (vx == 0 || vy == 0) ncc = 0.0;
    else {
        double x3 = (double)vx * (double)vy;
        double x4 = std::sqrt(x3);
        double c = (double)cov / x4;
        ncc = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    }
    double swr = 1.0 - ncc;
    double amm = (double)a / (256.0 * (double)B);
    double act = std::sqrt((amm + a0) * swr);
    out[0] = ncc; out[1] = swr; out[2] = amm; out[3] = act;
    return true;
}

// The best displacement of the 8 x 8 block of I at (x0, y0) among the
// candidates (cx, cy) + e, e in [-R, R]^2, against J read with clamp-to-edge:
// the smallest SAD, ties broken by the order of e (squared length, then ey,
// then ex).  With zero_mv only e = (0, 0) is a candidate.
void block_search(const Plane& I, const Plane& J, int x0, int y0, int cx, int cy, int R,
                  const std::vector<int>& rank, bool zero_mv, int& bdx, int& bdy, int& best_sad) {
    const int nc = 2 * R + 1;
    auto cJ = [&](int x, int y) {
        x = std::min(std::max(x, 0), J.w - 1);
        y = std::min(std::max(y, 0), J.h - 1);
        return J.at(x, y);
    };
    int best_rank = 0;
    best_sad = -1; bdx = cx; bdy = cy;
    for (int ey = -R; ey <= R; ++ey)
        for (int ex = -R; ex <= R; ++ex) {
            if (zero_mv && (ex != 0 || ey != 0)) continue;
            const int dx = cx + ex, dy = cy + ey;
            int s = 0;
            for (int j = 0; j < 8; ++j)
                for (int i = 0; i < 8; ++i)
                    s += std::abs(I.at(x0 + i, y0 + j) - cJ(x0 + i + dx, y0 + j + dy));
            const int r = rank[(size_t)(ey + R) * nc + (ex + R)];
            if (best_sad < 0 || s < best_sad || (s == best_sad && r < best_rank)) {
                best_sad = s; best_rank = r; bdx = dx; bdy = dy;
            }
        }
}

// The pair measure M(I -> J): for every whole 8 x 8 block of I a
// displacement d, J warped block-wise by those vectors, the exact moments of
// I against warped J over the covered pixels, and A = sum over blocks of
// floor(256 |d|).  The motion field (Sec. III.A) is
//  - full search: d in [-R, R]^2 minimising the SAD against J (clamp-to-edge),
//    ties broken by the candidate order; or, with hier,
//  - coarse-to-fine: I and J are box-downscaled once (the pyramid's own step),
//    each whole block of the coarse I gets its full-search vector d_c against
//    the coarse J; a block (bx, by) of I whose coarse block (bx/2, by/2) is
//    whole is predicted by 2 d_c, any other block by (0, 0); d is the best of
//    prediction + e, e in [-r, r]^2 against J, ties by the order of e.
//    Its reach is 2R + r per axis.
void pair_measure(const Plane& I, const Plane& J, const orc_params& p, bool zero_mv, bool hier, PairOut& o) {
    const int w = I.w, h = I.h, R = p.radius;
    o = PairOut();
    o.nbx = w / 8; o.nby = h / 8; o.B = (int64_t)o.nbx * o.nby;
    if (o.B <= 0 || J.w != w || J.h != h || R < 0 || (hier && p.refine < 0)) { o.ok = false; return; }
    auto cJ = [&](int x, int y) {
        x = std::min(std::max(x, 0), w - 1);
        y = std::min(std::max(y, 0), h - 1);
        return J.at(x, y);
    };
    o.mv.assign((size_t)o.B * 2, 0);
    o.sad.assign((size_t)o.B, 0);
    // predictions: (0, 0), or twice the coarse full-search vector
    std::vector<int> pred((size_t)o.B * 2, 0);
    if (hier && !zero_mv) {
        const Plane Ic = downscale(I), Jc = downscale(J);
        const int nbxc = Ic.w / 8, nbyc = Ic.h / 8;
        const std::vector<int> rankR = candidate_ranks(R);
        for (int by = 0; by < o.nby; ++by)
            for (int bx = 0; bx < o.nbx; ++bx) {
                if (bx / 2 >= nbxc || by / 2 >= nbyc) continue;
                int cdx, cdy, cs;
                block_search(Ic, Jc, 8 * (bx / 2), 8 * (by / 2), 0, 0, R, rankR, false, cdx, cdy, cs);
                const size_t b = (size_t)by * o.nbx + bx;
                pred[2 * b] = 2 * cdx; pred[2 * b + 1] = 2 * cdy;
            }
    }
    const int Rs = hier ? p.refine : R;
    const std::vector<int> rank = candidate_ranks(Rs);
    for (int by = 0; by < o.nby; ++by)
        for (int bx = 0; bx < o.nbx; ++bx) {
            const int x0 = 8 * bx, y0 = 8 * by;
            const size_t b = (size_t)by * o.nbx + bx;
            int bdx, bdy, best_sad;
            block_search(I, J, x0, y0, pred[2 * b], pred[2 * b + 1], Rs, rank, zero_mv, bdx, bdy, best_sad);
            o.mv[2 * b] = (int8_t)bdx; o.mv[2 * b + 1] = (int8_t)bdy;
            o.sad[b] = best_sad;
            for (int j = 0; j < 8; ++j)
                for (int i = 0; i < 8; ++i) {
                    const int64_t x = I.at(x0 + i, y0 + j);
                    const int64_t y = cJ(x0 + i + bdx, y0 + j + bdy);
                    o.sx += x; o.sy += y; o.sxx += x * x; o.syy += y * y; o.sxy += x * y;
                }
            o.a += isqrt64(65536 * (int64_t)(bdx * bdx + bdy * bdy));
        }
    o.n = 64 * o.B;
    o.is_static = o.a < (int64_t)p.a_static_fx * o.B;
    double f[4];
    if (!finish(o.sx, o.sy, o.sxx, o.syy, o.sxy, o.n, o.a, o.B, p.a0, f)) { o.ok = false; return; }
    o.ncc = f[0]; o.swr = f[1]; o.amm = f[2]; o.act = f[3];
}


// ---- Dense inverse search (search = 2): the paper's own kind of motion
// field (Sec. III.A names the dense inverse search optical flow of its
// reference [8]); this is a plain reading of that method on the same
// pyramid, with fixed work so that its result is exactly reproducible.
//
//  - Scales: the pair's two planes, then up to kDisScales box-downscaled
//    copies (the pyramid's own step), coarsest first; a copy narrower or
//    lower than one patch ends the list.
//  - Patches: kDisP x kDisP, origins every kDisS samples from 0, plus one
//    flush with the right (bottom) edge when the grid does not reach it.
//  - Per patch, inverse-compositional search: template T = the reference
//    patch, gradients by central differences over the whole plane (edge
//    samples repeated); H = sum g g^T + lambda I; kDisIters steps of
//    u <- u - H^-1 sum g (J(x + u) - T(x)), J sampled bilinearly with
//    clamp-to-edge coordinates; each component clamped to +-kDisUmax.
//    Start: 0 at the coarsest scale, else twice the coarser dense flow at
//    the patch centre halved (integer division, clamped).
//  - Densification: the flow at a pixel is the average of the vectors of the
//    patches covering it, weighted by 1 / max(1, |J(x + u) - I(x)|).
//  - Sums run in a fixed order (tree_sum): a patch's 64 terms in row-major
//    order are added as a balanced binary tree (pairs, then pairs of pairs);
//    a longer list (a row's pixels, then the rows' sums) is cut into runs of
//    64 (the last one filled with zeros), each run added as that tree and
//    the runs' sums added in order.
constexpr int kDisP = 8;
constexpr int kDisS = 4;
constexpr int kDisScales = 2;
constexpr int kDisIters = 8;
constexpr double kDisLambda = 64.0;
constexpr double kDisUmax = 32.0;

// Balanced binary tree sum of 64 terms: adjacent pairs, then adjacent pairs
// of those, and so on.
double tree64(const double* v) {
    double t[64];
    for (int i = 0; i < 64; ++i) t[i] = v[i];
    for (int step = 1; step < 64; step *= 2)
        for (int i = 0; i < 64; i += 2 * step) t[i] = t[i] + t[i + step];
    return t[0];
}

// Sum of n terms: runs of 64 (the last one filled with zeros) each added as a
// tree, the runs' sums added in order.
double tree_sum(const std::vector<double>& v) {
    double acc = 0.0;
    for (size_t c = 0; c < v.size(); c += 64) {
        double run[64];
        for (size_t i = 0; i < 64; ++i) run[i] = c + i < v.size() ? v[c + i] : 0.0;
        acc = acc + tree64(run);
    }
    return acc;
}

// Bilinear sample of J at (X, Y), coordinates clamped to the plane.
double bilin(const Plane& J, double X, double Y) {
    const double xc = std::min(std::max(X, 0.0), (double)(J.w - 1));
    const double yc = std::min(std::max(Y, 0.0), (double)(J.h - 1));
    const int x0 = (int)std::floor(xc), y0 = (int)std::floor(yc);
    const int x1 = std::min(x0 + 1, J.w - 1), y1 = std::min(y0 + 1, J.h - 1);
    const double fx = xc - x0, fy = yc - y0;
    const double a = J.at(x0, y0), b = J.at(x1, y0), c = J.at(x0, y1), d = J.at(x1, y1);
    const double top = a + fx * (b - a);
    const double bot = c + fx * (d - c);
    return top + fy * (bot - top);
}

std::vector<int> patch_origins(int n) {
    std::vector<int> o;
    for (int x = 0; x + kDisP <= n; x += kDisS) o.push_back(x);
    if (!o.empty() && o.back() + kDisP < n) o.push_back(n - kDisP);
    return o;
}

// Dense flow of I -> J (fx, fy per pixel of I, in the plane's pixels).
void dis_flow(const Plane& I0, const Plane& J0, std::vector<double>& fx, std::vector<double>& fy) {
    std::vector<Plane> Is{I0}, Js{J0};
    for (int k = 0; k < kDisScales; ++k) {
        Plane a = downscale(Is.back()), b = downscale(Js.back());
        if (a.w < kDisP || a.h < kDisP) break;
        Is.push_back(a);
        Js.push_back(b);
    }
    std::vector<double> cfx, cfy;        // the coarser scale's dense flow
    int cw = 0, ch = 0;
    for (int k = (int)Is.size() - 1; k >= 0; --k) {
        const Plane& I = Is[(size_t)k];
        const Plane& J = Js[(size_t)k];
        const int w = I.w, h = I.h;
        const std::vector<int> ox = patch_origins(w), oy = patch_origins(h);
        std::vector<double> ux(ox.size() * oy.size()), uy(ox.size() * oy.size());
        for (size_t j = 0; j < oy.size(); ++j)
            for (size_t i = 0; i < ox.size(); ++i) {
                const int px = ox[i], py = oy[j];
                double u0 = 0.0, u1 = 0.0;
                if (!cfx.empty()) {
                    const int cx = std::min((px + kDisP / 2) / 2, cw - 1);
                    const int cy = std::min((py + kDisP / 2) / 2, ch - 1);
                    u0 = 2.0 * cfx[(size_t)cy * cw + cx];
                    u1 = 2.0 * cfy[(size_t)cy * cw + cx];
                }
                double gx[kDisP * kDisP], gy[kDisP * kDisP], t0[kDisP * kDisP], t1[kDisP * kDisP],
                    t2[kDisP * kDisP];
                for (int y = 0; y < kDisP; ++y)
                    for (int x = 0; x < kDisP; ++x) {
                        const int X = px + x, Y = py + y, q = y * kDisP + x;
                        gx[q] = (I.at(std::min(X + 1, w - 1), Y) - I.at(std::max(X - 1, 0), Y)) / 2.0;
                        gy[q] = (I.at(X, std::min(Y + 1, h - 1)) - I.at(X, std::max(Y - 1, 0))) / 2.0;
                        t0[q] = gx[q] * gx[q];
                        t1[q] = gx[q] * gy[q];
                        t2[q] = gy[q] * gy[q];
                    }
                const double h00 = tree64(t0) + kDisLambda, h01 = tree64(t1), h11 = tree64(t2) + kDisLambda;
                const double det = h00 * h11 - h01 * h01;
                for (int it = 0; it < kDisIters; ++it) {
                    for (int y = 0; y < kDisP; ++y)
                        for (int x = 0; x < kDisP; ++x) {
                            const int X = px + x, Y = py + y, q = y * kDisP + x;
                            const double e = bilin(J, X + u0, Y + u1) - I.at(X, Y);
                            t0[q] = gx[q] * e;
                            t1[q] = gy[q] * e;
                        }
                    const double b0 = tree64(t0), b1 = tree64(t1);
                    const double d0 = (h11 * b0 - h01 * b1) / det;
                    const double d1 = (h00 * b1 - h01 * b0) / det;
                    u0 = std::min(std::max(u0 - d0, -kDisUmax), kDisUmax);
                    u1 = std::min(std::max(u1 - d1, -kDisUmax), kDisUmax);
                }
                ux[j * ox.size() + i] = u0;
                uy[j * ox.size() + i] = u1;
            }
        // densification
        std::vector<double> nfx((size_t)w * h), nfy((size_t)w * h);
        for (int Y = 0; Y < h; ++Y)
            for (int X = 0; X < w; ++X) {
                double n0 = 0.0, n1 = 0.0, den = 0.0;
                for (size_t j = 0; j < oy.size() && oy[j] <= Y; ++j) {      // origins ascend
                    if (oy[j] + kDisP <= Y) continue;
                    for (size_t i = 0; i < ox.size() && ox[i] <= X; ++i) {
                        if (ox[i] + kDisP <= X) continue;
                        const double u0 = ux[j * ox.size() + i], u1 = uy[j * ox.size() + i];
                        const double e = bilin(J, X + u0, Y + u1) - I.at(X, Y);
                        const double wgt = 1.0 / std::max(1.0, std::fabs(e));
                        n0 += wgt * u0;
                        n1 += wgt * u1;
                        den += wgt;
                    }
                }
                nfx[(size_t)Y * w + X] = n0 / den;
                nfy[(size_t)Y * w + X] = n1 / den;
            }
        cfx.swap(nfx);
        cfy.swap(nfy);
        cw = w;
        ch = h;
    }
    fx.swap(cfx);
    fy.swap(cfy);
}

// The pair measure with the dense flow: NCC of I against J warped by the
// flow (bilinear), over every pixel, AMM = mean flow magnitude, SWR, ACT;
// static if 256 AMM < a_static_fx (the block reading's threshold).
void flow_measure(const Plane& I, const Plane& J, const orc_params& p, PairOut& o, std::vector<double>* flow) {
    o = PairOut();
    const int w = I.w, h = I.h;
    if (w < kDisP || h < kDisP || J.w != w || J.h != h) { o.ok = false; return; }
    std::vector<double> fx, fy;
    dis_flow(I, J, fx, fy);
    // per row the six sums over its pixels, then the same over the rows
    std::vector<double> rows[6];
    for (int Y = 0; Y < h; ++Y) {
        std::vector<double> v[6];
        for (int X = 0; X < w; ++X) {
            const double u0 = fx[(size_t)Y * w + X], u1 = fy[(size_t)Y * w + X];
            const double x = I.at(X, Y);
            const double y = bilin(J, X + u0, Y + u1);
            v[0].push_back(x); v[1].push_back(y); v[2].push_back(x * x); v[3].push_back(y * y);
            v[4].push_back(x * y); v[5].push_back(std::sqrt(u0 * u0 + u1 * u1));
        }
        for (int k = 0; k < 6; ++k) rows[k].push_back(tree_sum(v[k]));
    }
    const double sx = tree_sum(rows[0]), sy = tree_sum(rows[1]), sxx = tree_sum(rows[2]);
    const double syy = tree_sum(rows[3]), sxy = tree_sum(rows[4]), sm = tree_sum(rows[5]);
    const double n = (double)w * h;
    const double cov = n * sxy - sx * sy;
    const double vx = n * sxx - sx * sx;
    const double vy = n * syy - sy * sy;
    double ncc;
    if (vx <= 0.0 && vy <= 0.0) ncc = 1.0;
    else if (vx <= 0.0 || vy <= 0.0) ncc = 0.0;
    else {
        const double c = cov / std::sqrt(vx * vy);
        ncc = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    }
    o.ncc = ncc;
    o.swr = 1.0 - ncc;
    o.amm = sm / n;
    o.act = std::sqrt((o.amm + p.a0) * o.swr);
    o.is_static = 256.0 * o.amm < (double)p.a_static_fx;
    o.n = (int64_t)w * h;
    if (flow) {
        flow->resize((size_t)2 * w * h);
        for (size_t i = 0; i < (size_t)w * h; ++i) { (*flow)[2 * i] = fx[i]; (*flow)[2 * i + 1] = fy[i]; }
    }
}

struct Meas { double act = 0, swr = 0; };

// Source of the pair measures used by the sequential pass.
struct Provider {
    virtual ~Provider() {}
    virtual bool consec(int t, orc_frame_rec& r) = 0;        // pair t -> t+1
    virtual bool field(int t, int which, Meas& m) = 0;        // v0, v1, v2
    virtual bool deepF(int t, int K, Meas& m) = 0;            // t -> t+K
    virtual bool deepP(int t, int K, int Kp, Meas& m) = 0;    // t -> t-Kp at the level of K
    virtual void evict_before(int) {}
    std::vector<orc_measure_key> log;
};

// Sampling-structure vote over the analysed frames of one shot (Sec. III.C).
struct Analysis {
    bool open = true;
    int n = 0, nci = 0, s = 0, result = 0, phase = -1;
    int np[5] = {0, 0, 0, 0, 0};
    double s0[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double sum1 = 0.0, sum2 = 0.0;

    // Interlace vote, one reading of "v0 is not near zero" (Sec. III.C): v0
    // against the smaller inter-frame field activity.  In interlaced content
    // v0 and one of v1/v2 span half a frame interval, so v0 is comparable to
    // min(v1, v2) even when the other pair moves too far for the search
    // range; in progressive content v1 and v2 span a full interval and v0
    // none.  For the 3:2 pulldown cadence v0 is summed per position of the
    // 5-frame pulldown unit (phase = frame index in the shot mod 5).
    void add(int ph, double v0, double v1, double v2, const orc_params& p) {
        const bool comb_min = v0 > p.tau_c * std::min(v1, v2);
        ++n; ++np[ph];
        if (comb_min) ++nci;
        s0[ph] = s0[ph] + v0;
        if (v1 > v2) ++s; else if (v1 < v2) --s;
        sum1 = sum1 + v1; sum2 = sum2 + v2;
    }
    // Mean v0 at position a exceeds tau_p times the mean at position r
    // (cross-multiplied, so no division is rounded).
    bool dominates(int a, int r, const orc_params& p) const {
        return s0[a] * (double)np[r] > p.tau_p * (s0[r] * (double)np[a]);
    }
    void decide(const orc_params& p) {
        open = false;
        phase = -1;
        if (n == 0) { result = 0; return; }
        if (n >= 10 && np[0] && np[1] && np[2] && np[3] && np[4]) {
            // 3:2 pulldown: the frames whose two fields come from different
            // film frames (the combed ones) sit at two neighbouring positions
            // q, q+1 of the unit; their mean v0 exceeds tau_p times the mean
            // at each of the other three positions.  With tau_p >= 1 at most
            // one q qualifies.
            for (int q = 0; q < 5; ++q) {
                const int a = q, b = (q + 1) % 5;
                bool ok = true;
                for (int r = 0; r < 5 && ok; ++r)
                    if (r != a && r != b) ok = dominates(a, r, p) && dominates(b, r, p);
                if (ok) { result = 4; phase = q; return; }
            }
        }
        bool inter;
        if ((double)nci <= p.eps * (double)n) inter = false;
        else if ((double)nci >= (1.0 - p.eps) * (double)n) inter = true;
        else inter = 2 * nci > n;
        if (!inter) { result = 1; return; }
        // Field order from beta = v1 / v2: > 1 upper field first, < 1 lower first.
        if (s > 0) result = 2;
        else if (s < 0) result = 3;
        else result = (sum1 >= sum2) ? 2 : 3;
    }
};

// Deep check at frame t (Sec. III.B): a K-frame transition after t is accepted
// when the activity from t to t+K clearly exceeds the activity from t back to
// its predecessor at the same distance; K and K+1 must both verify (a single
// odd frame such as a flash verifies only one).  Among the candidates the
// first whose excess activity E_K = ACT(t, t+K) - ACT(t, t-K) reaches gamma
// of the largest one is taken: both activities are measured at the same
// distance and pyramid level, so E_K stops growing once t+K lies in the new
// shot, where a plain dissimilarity keeps growing with K.
bool deep_check(int t, int T, int shot_start, double a_t, double s_t, Provider& pv,
                const orc_params& p, int& Kstar) {
    Kstar = 0;
    const int Kn = std::min(p.k_max + 1, T - 1 - t);
    std::vector<char> V((size_t)p.k_max + 3, 1);
    std::vector<double> S((size_t)p.k_max + 3, 0.0);
    for (int K = 1; K <= Kn; ++K) {
        Meas f;
        if (K == 1) { f.act = a_t; f.swr = s_t; }
        else if (!pv.deepF(t, K, f)) return false;
        const int Kp = std::min(K, t - shot_start);
        double pa = 0.0;
        if (Kp > 0) { Meas b; if (!pv.deepP(t, K, Kp, b)) return false; pa = b.act; }
        V[K] = f.act > p.rho_d * pa + p.theta_d;
        S[K] = f.act - pa;
    }
    const int Kc = std::min(p.k_max, Kn);
    bool any = false;
    double smax = 0.0;
    for (int K = 1; K <= Kc; ++K)
        if (V[K] && V[K + 1]) { if (!any || S[K] > smax) smax = S[K]; any = true; }
    if (!any) return true;
    for (int K = 1; K <= Kc; ++K)
        if (V[K] && V[K + 1] && S[K] >= p.gamma * smax) { Kstar = K; return true; }
    return true;
}

void init_record(orc_frame_rec& r, int64_t f) {
    std::memset(&r, 0, sizeof r);
    r.frame = f;
    r.shot_id = -1;
    const double nan = std::nan("");
    r.ncc = r.swr = r.amm = r.act = nan;
    r.v[0] = r.v[1] = r.v[2] = nan;
    r.h_mean = r.h_std = r.h_mad = nan;
}

// Sec. III.A: H(t), the intensity histogram of a frame, and its mean,
// standard deviation and mean absolute deviation.  The sums are exact
// integers; each measure is rounded once:
//   mean = S1 / N,  std = sqrt(N S2 - S1^2) / N,  mad = sum_v h[v] |N v - S1| / N^2,
// which are sum(x)/N, sqrt(sum((x - mean)^2) / N) and sum(|x - mean|) / N
// with the sums taken exactly.
struct Intensity {
    std::vector<int64_t> h;
    int64_t n = 0, s1 = 0, s2 = 0, m = 0;
    double mean = 0, sd = 0, mad = 0;
};

Intensity intensity(const Plane& q, int bits) {
    Intensity o;
    o.h.assign((size_t)1 << bits, 0);
    for (int32_t v : q.px) o.h[(size_t)v] += 1;
    for (size_t v = 0; v < o.h.size(); ++v) {
        o.n += o.h[v];
        o.s1 += (int64_t)v * o.h[v];
        o.s2 += (int64_t)v * (int64_t)v * o.h[v];
    }
    for (size_t v = 0; v < o.h.size(); ++v) {
        const int64_t d = o.n * (int64_t)v - o.s1;
        o.m += o.h[v] * (d < 0 ? -d : d);
    }
    const __int128 var_n2 = (__int128)o.n * o.s2 - (__int128)o.s1 * o.s1;   // N^2 times the variance
    o.mean = (double)o.s1 / (double)o.n;
    o.sd = std::sqrt((double)var_n2) / (double)o.n;
    o.mad = (double)o.m / ((double)o.n * (double)o.n);
    return o;
}

// The offline sequential pass: one iteration per frame t, jumping over a
// detected transition.
int run_pass(int T, Provider& pv, const orc_params& p, bool dense,
             std::vector<orc_frame_rec>& recs, std::vector<orc_shot_rec>& shots) {
    recs.assign((size_t)T, orc_frame_rec());
    for (int f = 0; f < T; ++f) init_record(recs[(size_t)f], f);
    shots.clear();
    if (T <= 0) return 0;
    int done = -1;  // consecutive pairs are computed for every frame, in order
    auto ensure = [&](int upto) {
        while (done < upto) { ++done; if (!pv.consec(done, recs[(size_t)done])) return false; }
        return true;
    };
    recs[0].flags |= ORC_F_KEYFRAME | ORC_F_SHOT_START;
    orc_shot_rec cur;
    std::memset(&cur, 0, sizeof cur);
    cur.pulldown_phase = -1;
    int shot_start = 0, shot_id = 0;
    std::deque<double> hist;
    double acc = 0.0;
    Analysis ss;
    auto close_shot = [&](int last) {
        if (ss.open) ss.decide(p);
        cur.last = last;
        cur.sampling = ss.result;
        cur.pulldown_phase = ss.result == 4 ? ss.phase : -1;
        cur.n_analyzed = ss.n;
        cur.final_ = 1;
        shots.push_back(cur);
    };
    int t = 0;
    while (t < T - 1) {
        pv.evict_before(t - p.k_max - 2);
        if (!ensure(t)) return -1;
        orc_frame_rec& r = recs[(size_t)t];
        const double a = r.act;
        const bool st = (r.flags & ORC_F_STATIC) != 0;
        const bool want_fields = ss.open && !st;   // static frames carry no information
        if (want_fields || dense) {
            Meas v[3];
            for (int i = 0; i < 3; ++i) if (!pv.field(t, i, v[i])) return -1;
            if (want_fields) {
                for (int i = 0; i < 3; ++i) r.v[i] = v[i].act;
                r.field_mask = 7;
                r.flags |= ORC_F_ANALYZED;
                ss.add((t - shot_start) % 5, v[0].act, v[1].act, v[2].act, p);
                if (ss.n == p.n_ss) ss.decide(p);
            }
        }
        // Fast check against the recent activity of the current shot.
        double thr;
        if (hist.empty()) thr = p.theta_f0;       // no history yet: absolute threshold
        else {
            double s = 0.0;
            for (double x : hist) s = s + x;
            const double mean = s / (double)hist.size();
            thr = p.rho_f * mean + p.theta_f;
        }
        const bool fire = a > thr;
        if (fire) r.flags |= ORC_F_FAST_FIRED;
        int Kstar = 0;
        if (fire || dense) {
            if (!ensure(std::min(T - 2, t + p.k_max + 1))) return -1;
            if (!deep_check(t, T, shot_start, a, r.swr, pv, p, Kstar)) return -1;
            if (!fire) Kstar = 0;
        }
        if (Kstar > 0) {
            close_shot(t);
            for (int f = t + 1; f < t + Kstar; ++f) recs[(size_t)f].flags |= ORC_F_IN_TRANSITION;
            const int b = t + Kstar;
            orc_frame_rec& rb = recs[(size_t)b];
            rb.boundary = Kstar == 1 ? 1 : 2;
            rb.boundary_k = Kstar;
            rb.flags |= ORC_F_SHOT_START | ORC_F_KEYFRAME;
            ++shot_id;
            std::memset(&cur, 0, sizeof cur);
            cur.shot_id = shot_id;
            cur.first = b;
            cur.in_boundary = rb.boundary;
            cur.in_k = Kstar;
            cur.pulldown_phase = -1;
            shot_start = b;
            hist.clear();
            acc = 0.0;
            ss = Analysis();
            t = b;
            continue;
        }
        // The history takes the activity capped at the threshold, so that a
        // flash or other one-off spike does not mask what follows it.
        hist.push_back(fire ? thr : a);
        if ((int)hist.size() > p.w_hist) hist.pop_front();
        // Dynamic keyframes: accumulate consecutive-frame activity within the shot.
        acc = acc + a;
        if (acc > p.theta_kf) { recs[(size_t)t + 1].flags |= ORC_F_KEYFRAME; acc = 0.0; }
        ++t;
    }
    if (!ensure(T - 2)) return -1;
    close_shot(T - 1);
    for (const orc_shot_rec& s : shots)
        for (int64_t f = s.first; f <= s.last; ++f) recs[(size_t)f].shot_id = s.shot_id;
    return 0;
}

void fill_pair_record(orc_frame_rec& r, const PairOut& o) {
    r.flags |= ORC_F_HAS_PAIR;
    if (o.is_static) r.flags |= ORC_F_STATIC;
    r.ncc = o.ncc; r.swr = o.swr; r.amm = o.amm; r.act = o.act;
    r.mom[0] = o.sx; r.mom[1] = o.sy; r.mom[2] = o.sxx; r.mom[3] = o.syy; r.mom[4] = o.sxy;
    r.n_pix = o.n; r.amm_num = o.a; r.n_blocks = (int32_t)o.B;
}

typedef std::tuple<int, int, int, int, int> Key;  // ref, ref_field, oth, oth_field, level

// Measures computed from frames, on demand, each at most once.
struct FrameProvider : Provider {
    const unsigned char* base;
    int T;
    int64_t pitch, stride;
    int bits;
    Geometry g;
    orc_params p;
    int8_t* mv_out;
    std::map<int, FrameLevels> levels;
    std::map<Key, Meas> cache;
    bool bad_input = false;

    const FrameLevels* get(int f) {
        auto it = levels.find(f);
        if (it != levels.end()) return &it->second;
        Plane full;
        if (!load_frame(base + (size_t)f * (size_t)stride, g.W, g.H, pitch, bits, full)) {
            bad_input = true;
            return nullptr;
        }
        FrameLevels& fl = levels[f];
        build_levels(full, g, fl);
        return &fl;
    }
    const Plane& plane(const FrameLevels& fl, int field, int level) {
        if (field == 1) return fl.U;
        if (field == 2) return fl.Dc;
        return fl.lv[(size_t)(level - g.L)];
    }
    bool measure(int kind, int ref, int rf, int oth, int of, int level, Meas& m, PairOut* keep) {
        Key k(ref, rf, oth, of, level);
        auto it = cache.find(k);
        if (it != cache.end() && !keep) { m = it->second; return true; }
        const FrameLevels* a = get(ref);
        const FrameLevels* b = get(oth);
        if (!a || !b) return false;
        PairOut o;
        // search 2: the dense flow for every pair; else field pairs keep the
        // full search and frame pairs follow p.search
        if (p.search == 2) flow_measure(plane(*a, rf, level), plane(*b, of, level), p, o, nullptr);
        else pair_measure(plane(*a, rf, level), plane(*b, of, level), p, false, p.search == 1 && kind != 1, o);
        if (!o.ok) return false;
        m.act = o.act; m.swr = o.swr;
        if (it == cache.end()) {
            cache[k] = m;
            log.push_back(orc_measure_key{kind, ref, oth, rf, of, level});
        }
        if (keep) *keep = o;
        return true;
    }
    bool consec(int t, orc_frame_rec& r) override {
        PairOut o;
        Meas m;
        if (!measure(0, t, 0, t + 1, 0, g.L, m, &o)) return false;
        fill_pair_record(r, o);
        if (mv_out && !o.mv.empty()) std::memcpy(mv_out + (size_t)t * o.mv.size(), o.mv.data(), o.mv.size());
        return true;
    }
    bool field(int t, int which, Meas& m) override {
        // v0: U_t -> D_t, v1: U_t -> D_{t+1}, v2: D_t -> U_{t+1}
        if (which == 0) return measure(1, t, 1, t, 2, g.Lf, m, nullptr);
        if (which == 1) return measure(1, t, 1, t + 1, 2, g.Lf, m, nullptr);
        return measure(1, t, 2, t + 1, 1, g.Lf, m, nullptr);
    }
    bool deepF(int t, int K, Meas& m) override {
        return measure(2, t, 0, t + K, 0, deep_level(g, K), m, nullptr);
    }
    bool deepP(int t, int K, int Kp, Meas& m) override {
        return measure(3, t, 0, t - Kp, 0, deep_level(g, K), m, nullptr);
    }
    void evict_before(int f) override {
        while (!levels.empty() && levels.begin()->first < f) levels.erase(levels.begin());
    }
};

// Measures read from injected sequences (decision logic alone).
struct InjectedProvider : Provider {
    int T, kw;
    const double *act, *swr, *v, *F, *S, *P;
    const uint8_t* stat;
    bool consec(int t, orc_frame_rec& r) override {
        r.flags |= ORC_F_HAS_PAIR;
        if (stat[t]) r.flags |= ORC_F_STATIC;
        r.act = act[t]; r.swr = swr[t]; r.ncc = 1.0 - swr[t];
        log.push_back(orc_measure_key{0, t, t + 1, 0, 0, 0});
        return true;
    }
    bool field(int t, int which, Meas& m) override {
        m.act = v[(size_t)t * 3 + which]; m.swr = 0.0;
        const int ref_f = which == 2 ? 2 : 1, oth_f = which == 2 ? 1 : 2;
        log.push_back(orc_measure_key{1, t, which == 0 ? t : t + 1, ref_f, oth_f, -1});
        return true;
    }
    bool deepF(int t, int K, Meas& m) override {
        m.act = F[(size_t)t * kw + K]; m.swr = S[(size_t)t * kw + K];
        log.push_back(orc_measure_key{2, t, t + K, 0, 0, ceil_log2(K)});
        return true;
    }
    // The backward pair t -> t-Kp at a given level is one measure, whatever K
    // asked for it: the first value requested stands (as with real frames).
    std::map<std::tuple<int, int, int>, double> pcache;
    bool deepP(int t, int K, int Kp, Meas& m) override {
        const auto key = std::make_tuple(t, t - Kp, ceil_log2(K));
        auto it = pcache.find(key);
        m.swr = 0.0;
        if (it != pcache.end()) { m.act = it->second; return true; }
        m.act = P[(size_t)t * kw + K];
        pcache[key] = m.act;
        log.push_back(orc_measure_key{3, t, t - Kp, 0, 0, ceil_log2(K)});
        return true;
    }
};

bool params_ok(const orc_params* p) {
    return p && p->block == 8 && p->radius >= 0 && p->radius <= 16 && p->k_max >= 1 &&
           p->k_max <= 64 && p->w_hist >= 1 && p->n_ss >= 1 && p->lf_offset >= 0 && p->tau_p >= 1.0 &&
           p->search >= 0 && p->search <= 2 && p->refine >= 0 && 2 * p->radius + p->refine <= 127;
}

int export_results(const std::vector<orc_frame_rec>& recs, const std::vector<orc_shot_rec>& shots,
                   const std::vector<orc_measure_key>& log, orc_frame_rec* out, orc_shot_rec* sh,
                   int32_t shots_cap, int32_t* n_shots, orc_measure_key* keys, int32_t keys_cap,
                   int32_t* n_keys) {
    if (out && !recs.empty()) std::memcpy(out, recs.data(), recs.size() * sizeof(orc_frame_rec));
    if (n_shots) *n_shots = (int32_t)shots.size();
    if (n_keys) *n_keys = (int32_t)log.size();
    if (sh) {
        if ((int64_t)shots.size() > shots_cap) return -3;
        if (!shots.empty()) std::memcpy(sh, shots.data(), shots.size() * sizeof(orc_shot_rec));
    }
    if (keys) {
        if ((int64_t)log.size() > keys_cap) return -3;
        if (!log.empty()) std::memcpy(keys, log.data(), log.size() * sizeof(orc_measure_key));
    }
    return 0;
}

}  // namespace

extern "C" {

int32_t orc_geometry(int32_t W, int32_t H, const orc_params* p, int32_t* out, int32_t cap) {
    if (!params_ok(p) || !out) return -1;
    Geometry g;
    if (!make_geometry(W, H, *p, g)) return -1;
    const int need = 4 + 2 * (g.Lcap + 1) + 2;
    if (cap < need) return -3;
    out[0] = g.L; out[1] = g.Lcap; out[2] = g.Lf; out[3] = g.Lcap + 1;
    for (int l = 0; l <= g.Lcap; ++l) { out[4 + 2 * l] = g.wl[l]; out[5 + 2 * l] = g.hl[l]; }
    out[4 + 2 * (g.Lcap + 1)] = g.wf;
    out[5 + 2 * (g.Lcap + 1)] = g.hf;
    return 0;
}

int32_t orc_downscale(const uint16_t* src, int32_t w, int32_t h, uint16_t* dst) {
    if (!src || !dst || w < 2 || h < 2) return -1;
    Plane s;
    s.w = w; s.h = h;
    s.px.assign(src, src + (size_t)w * h);
    Plane d = downscale(s);
    for (size_t i = 0; i < d.px.size(); ++i) dst[i] = (uint16_t)d.px[i];
    return 0;
}

int32_t orc_levels(const void* Y, int32_t W, int32_t H, int64_t pitch_bytes, int32_t bits,
                   const orc_params* p, uint16_t* out, int64_t cap, int64_t* n_out) {
    if (!Y || !params_ok(p) || (bits != 8 && bits != 10)) return -1;
    Geometry g;
    if (!make_geometry(W, H, *p, g)) return -1;
    if (pitch_bytes < (int64_t)W * (bits == 8 ? 1 : 2)) return -1;
    Plane full;
    if (!load_frame(Y, W, H, pitch_bytes, bits, full)) return -1;
    FrameLevels fl;
    build_levels(full, g, fl);
    int64_t n = 0;
    for (const Plane& q : fl.lv) n += (int64_t)q.px.size();
    n += (int64_t)fl.U.px.size() + (int64_t)fl.D.px.size() + (int64_t)fl.Dc.px.size();
    if (n_out) *n_out = n;
    if (!out) return 0;
    if (cap < n) return -3;
    int64_t k = 0;
    auto put = [&](const Plane& q) { for (int32_t v : q.px) out[k++] = (uint16_t)v; };
    for (const Plane& q : fl.lv) put(q);
    put(fl.U);
    put(fl.D);
    put(fl.Dc);
    return 0;
}

int32_t orc_pair(const uint16_t* I, const uint16_t* J, int32_t w, int32_t h, const orc_params* p,
                 int32_t force_zero_mv, int8_t* mv, int32_t* sad, int64_t* ints, double* dbl) {
    if (!I || !J || !params_ok(p) || w < 8 || h < 8) return -1;
    Plane a, b;
    a.w = b.w = w; a.h = b.h = h;
    a.px.assign(I, I + (size_t)w * h);
    b.px.assign(J, J + (size_t)w * h);
    PairOut o;
    pair_measure(a, b, *p, force_zero_mv != 0, p->search == 1, o);
    if (!o.ok) return -1;
    if (mv) std::memcpy(mv, o.mv.data(), o.mv.size());
    if (sad) std::memcpy(sad, o.sad.data(), o.sad.size() * sizeof(int32_t));
    if (ints) {
        int64_t v[9] = {o.sx, o.sy, o.sxx, o.syy, o.sxy, o.n, o.a, o.B, o.is_static ? 1 : 0};
        std::memcpy(ints, v, sizeof v);
    }
    if (dbl) { dbl[0] = o.ncc; dbl[1] = o.swr; dbl[2] = o.amm; dbl[3] = o.act; }
    return 0;
}

int32_t orc_flow_pair(const uint16_t* I, const uint16_t* J, int32_t w, int32_t h, const orc_params* p,
                      double* flow, double* dbl, int32_t* is_static) {
    if (!I || !J || !params_ok(p) || w < kDisP || h < kDisP) return -1;
    Plane a, b;
    a.w = b.w = w; a.h = b.h = h;
    a.px.assign(I, I + (size_t)w * h);
    b.px.assign(J, J + (size_t)w * h);
    PairOut o;
    std::vector<double> f;
    flow_measure(a, b, *p, o, flow ? &f : nullptr);
    if (!o.ok) return -1;
    if (flow) std::memcpy(flow, f.data(), f.size() * sizeof(double));
    if (dbl) { dbl[0] = o.ncc; dbl[1] = o.swr; dbl[2] = o.amm; dbl[3] = o.act; }
    if (is_static) *is_static = o.is_static ? 1 : 0;
    return 0;
}

int32_t orc_finish(const int64_t* v, double a0, double* out4) {
    if (!v || !out4) return -1;
    return finish(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], a0, out4) ? 0 : -1;
}

int32_t orc_run_clip(const void* frames, int32_t T, int32_t W, int32_t H, int64_t pitch_bytes,
                     int64_t frame_stride_bytes, int32_t bits, int32_t dense, const orc_params* p,
                     orc_frame_rec* recs, orc_shot_rec* shots, int32_t shots_cap, int32_t* n_shots,
                     orc_measure_key* keys, int32_t keys_cap, int32_t* n_keys, int8_t* mv_out) {
    if (!frames || T < 1 || !params_ok(p) || (bits != 8 && bits != 10)) return -1;
    FrameProvider pv;
    if (!make_geometry(W, H, *p, pv.g)) return -1;
    const int64_t row = (int64_t)W * (bits == 8 ? 1 : 2);
    if (pitch_bytes < row || frame_stride_bytes < pitch_bytes * (H - 1) + row) return -1;
    pv.base = (const unsigned char*)frames;
    pv.T = T; pv.pitch = pitch_bytes; pv.stride = frame_stride_bytes; pv.bits = bits;
    pv.p = *p; pv.mv_out = mv_out;
    std::vector<orc_frame_rec> r;
    std::vector<orc_shot_rec> s;
    if (run_pass(T, pv, *p, dense != 0, r, s) != 0) return -1;
    // the unary measure of every frame, over its working-level image
    for (int t = 0; t < T; ++t) {
        const FrameLevels* fl = pv.get(t);
        if (!fl) return -1;
        const Intensity in = intensity(fl->lv[0], bits);
        r[(size_t)t].h_mean = in.mean;
        r[(size_t)t].h_std = in.sd;
        r[(size_t)t].h_mad = in.mad;
    }
    return export_results(r, s, pv.log, recs, shots, shots_cap, n_shots, keys, keys_cap, n_keys);
}

int32_t orc_intensity(const uint16_t* px, int32_t w, int32_t h, int32_t bits, int64_t* hist, int64_t* ints,
                      double* out3) {
    if (!px || w < 1 || h < 1 || (bits != 8 && bits != 10)) return -1;
    Plane q;
    q.w = w; q.h = h;
    q.px.assign(px, px + (size_t)w * h);
    for (int32_t v : q.px) if (v >= (1 << bits)) return -1;
    const Intensity in = intensity(q, bits);
    if (hist) std::memcpy(hist, in.h.data(), in.h.size() * sizeof(int64_t));
    if (ints) { ints[0] = in.n; ints[1] = in.s1; ints[2] = in.s2; ints[3] = in.m; }
    if (out3) { out3[0] = in.mean; out3[1] = in.sd; out3[2] = in.mad; }
    return 0;
}

int32_t orc_decide_injected(int32_t T, const double* act, const double* swr, const uint8_t* stat,
                            const double* v, const double* F, const double* S, const double* P,
                            int32_t dense, const orc_params* p, orc_frame_rec* recs,
                            orc_shot_rec* shots, int32_t shots_cap, int32_t* n_shots,
                            orc_measure_key* keys, int32_t keys_cap, int32_t* n_keys) {
    if (T < 1 || !act || !swr || !stat || !v || !F || !S || !P || !params_ok(p)) return -1;
    InjectedProvider pv;
    pv.T = T; pv.kw = p->k_max + 2;
    pv.act = act; pv.swr = swr; pv.stat = stat; pv.v = v; pv.F = F; pv.S = S; pv.P = P;
    std::vector<orc_frame_rec> r;
    std::vector<orc_shot_rec> s;
    if (run_pass(T, pv, *p, dense != 0, r, s) != 0) return -1;
    return export_results(r, s, pv.log, recs, shots, shots_cap, n_shots, keys, keys_cap, n_keys);
}

}  // extern "C"
