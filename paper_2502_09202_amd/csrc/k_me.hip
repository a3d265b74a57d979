// k_me.hip -- K2: block motion search + warped moments, K3: pair finish.
//
// Pair measure of I -> J at one pyramid level (the reading of Sec. III.A used
// here): for every whole 8x8 block of I, the displacement d in [-8, 8]^2 with
// the smallest SAD against J (J read clamp-to-edge); ties go to the candidate
// first in the order (|d|^2, dy, dx).  J is warped block-wise by d; the exact
// moments Sx, Sy, Sxx, Syy, Sxy of I against warped J over the covered pixels
// and A = sum_b floor(256 |d_b|) give NCC, SWR = 1 - NCC, AMM = A / (256 B) and
// ACT = sqrt((AMM + a0) SWR).
//
// K2 layout: one 256-thread workgroup per tile of 8 x 8 blocks (64 x 64
// pixels of I).  The tile of I and its (64+16) x (64+16) search window of J
// are staged in LDS once (clamped at the plane edges), so every candidate is
// read from LDS.  Four lanes share a block: lane q searches dy in
// [-8+4q, -5+4q] over all dx and one quarter of the dy = +8 row.
// 8-bit: v_qsad_pk_u16_u8 gives the SADs of four consecutive dx from one
// aligned 8-byte window (dx groups -8, -4, 0, +4), v_sad_u8 covers dx = +8, so
// no byte alignment is ever needed in the search loop; each J row a lane needs
// is read from LDS once and used for all four of its dy.  10-bit: v_sad_u16 on
// pairs of samples with a 2-byte realignment for odd dx.  Each candidate's key
// is (SAD << 16) + code(dx, dy), where the code is strictly increasing in the
// candidate order (|d|^2, dy, dx) and below 2^16, so the minimum key is the
// unique argmin; the code is arithmetic, no table is read.  The epilogue reads the warped block from the same
// LDS window and forms int32 moments per lane, reduced per tile to int64.
// K3 sums the tile partials of each pair and forms the doubles in a fixed
// order with no contraction.
#include "vsa_internal.h"
#include "pair_finish.h"

namespace vsa {

namespace {

// Tie-break code of candidate (dx, dy): ((dx^2 + dy^2) * 17 + dy + 8) * 17 +
// dx + 8, the candidate's position in mixed radix, so codes increase strictly
// in the order (|d|^2, dy, dx); at most 128 * 289 + 288 < 2^16.  Split into a
// dx part and a dy part that add up to it.
__host__ __device__ constexpr uint32_t code_dx(int dx) { return (uint32_t)(dx * dx * 289 + dx + 8); }
__host__ __device__ constexpr uint32_t code_dy(int dy) { return (uint32_t)(dy * dy * 289 + (dy + 8) * 17); }
static_assert(code_dx(8) + code_dy(8) < 65536u, "candidate code must fit 16 bits");

constexpr int kJW8 = 80;   // J window row length (bytes, 8-bit)
constexpr int kXcd = 8;    // accelerator complex dies, one L2 each
constexpr int kJRows = 80;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

struct PlaneRef {
    const uint8_t* base;
    int w, h, pitch;   // pitch in samples
    int cosite;        // 0, or s = Lf + 1: read the lower field on the upper field's rows
};

__device__ __forceinline__ PlaneRef plane_of(const StreamDesc& sd, int frame, int field, int level) {
    PlaneRef p;
    const uint8_t* slot = sd.ring + (int64_t)(frame % sd.rs) * sd.slot_bytes;
    if (field == PL_UPPER || field == PL_LOWER) {
        p.base = slot + (field == PL_UPPER ? sd.offU : sd.offD);
        p.w = sd.wf; p.h = sd.hf; p.pitch = sd.pf;
        p.cosite = field == PL_LOWER ? sd.Lf + 1 : 0;
    } else {
        const int d = level - sd.L;
        p.base = slot + sd.off[d];
        p.w = sd.wl[d]; p.h = sd.hl[d]; p.pitch = sd.pl[d];
        p.cosite = 0;
    }
    return p;
}

// floor(256 * sqrt(m)) for 0 <= m <= 128, exact.
__device__ __forceinline__ int amm_fx(int m) {
    const int v = 65536 * m;
    int r = (int)__builtin_sqrtf((float)v);
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// The lower field on the upper field's rows.  Both fields have a row pitch of
// p = 2^s full-resolution rows (s = Lf + 1) and the lower field lies one
// full-resolution row lower, so row y of the resampled plane is
// ((p-1) D[y] + D[y-1] + p/2) >> s, with D[-1] read as D[0].  Field pairs read
// the lower field only through this (an integer motion field cannot absorb
// the sub-row offset between the fields).
template <typename T, typename V>
__device__ __forceinline__ V cosite_vec(V a, V b, int s) {
    constexpr int N = (int)(sizeof(V) / sizeof(T));
    union U { V v; T t[N]; };
    U ua, ub, uo;
    ua.v = a;
    ub.v = b;
    const int p = 1 << s;
#pragma unroll
    for (int k = 0; k < N; ++k) uo.t[k] = (T)(((p - 1) * (int)ua.t[k] + (int)ub.t[k] + (p >> 1)) >> s);
    return uo.v;
}

template <typename T>
__device__ __forceinline__ void stage_I(const PlaneRef& P, int bx0, int by0, uint8_t* sI) {
    // I tile: 64 rows x 64 samples.  The tile origin is a multiple of 64
    // samples inside the row, so each 16-byte chunk lies within the row pitch;
    // rows past the plane are clamped (they feed no block).
    constexpr int B = (int)sizeof(T);
    constexpr int CH = 64 * B / 16;
    for (int i = threadIdx.x; i < 64 * CH; i += kMEThreads) {
        const int r = i / CH, c = i % CH;
        const int gy = clampi(8 * by0 + r, 0, P.h - 1);
        const uint4* src = reinterpret_cast<const uint4*>(P.base + ((int64_t)gy * P.pitch + 8 * bx0) * B) + c;
        uint4 v = *src;
        if (P.cosite) {
            const int gp = gy > 0 ? gy - 1 : 0;
            const uint4* prv = reinterpret_cast<const uint4*>(P.base + ((int64_t)gp * P.pitch + 8 * bx0) * B) + c;
            v = cosite_vec<T, uint4>(v, *prv, P.cosite);
        }
        reinterpret_cast<uint4*>(sI + r * 64 * B)[c] = v;
    }
}

template <typename T>
__device__ __forceinline__ void stage_J(const PlaneRef& P, int bx0, int by0, uint8_t* sJ) {
    // J window: rows 8*by0-8 .. +80, columns 8*bx0-8 .. +80, clamped to the plane.
    constexpr int B = (int)sizeof(T);
    constexpr int CH = kJW8 * B / 8;                 // 8-byte chunks per row
    const int x0 = 8 * bx0 - 8;
    for (int i = threadIdx.x; i < kJRows * CH; i += kMEThreads) {
        const int r = i / CH, c = i % CH;
        const int gy = clampi(8 * by0 - 8 + r, 0, P.h - 1);
        const int gx = x0 + c * (8 / B);
        const T* row = reinterpret_cast<const T*>(P.base + (int64_t)gy * P.pitch * B);
        const T* prv = reinterpret_cast<const T*>(P.base + (int64_t)(gy > 0 ? gy - 1 : 0) * P.pitch * B);
        uint2 v, w = make_uint2(0u, 0u);
        if (gx >= 0 && gx + 8 / B <= P.w) {
            v = *reinterpret_cast<const uint2*>(row + gx);
            if (P.cosite) w = *reinterpret_cast<const uint2*>(prv + gx);
        } else {
            union { T t[8 / B]; uint2 u; } tmp, tmq;
#pragma unroll
            for (int k = 0; k < 8 / B; ++k) {
                tmp.t[k] = row[clampi(gx + k, 0, P.w - 1)];
                tmq.t[k] = P.cosite ? prv[clampi(gx + k, 0, P.w - 1)] : (T)0;
            }
            v = tmp.u;
            w = tmq.u;
        }
        if (P.cosite) v = cosite_vec<T, uint2>(v, w, P.cosite);
        *reinterpret_cast<uint2*>(sJ + r * kJW8 * B + c * 8) = v;
    }
}

__device__ __forceinline__ uint64_t pk64(uint32_t lo, uint32_t hi) {
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// 8-bit search for one lane: returns the best key (SAD << 16) + code(dx, dy).
// The lane's four dy rows are visited one at a time (eight J rows each, read
// from LDS), which keeps only five accumulators live; register pressure, not
// LDS bandwidth, is what limits this kernel's occupancy.
__device__ __forceinline__ uint32_t search8(const uint8_t* sI, const uint8_t* sJ, int bx, int by, int q) {
    uint32_t r0[8], r1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint2 v = *reinterpret_cast<const uint2*>(sI + (8 * by + j) * 64 + 8 * bx);
        r0[j] = v.x;
        r1[j] = v.y;
    }
    uint32_t best = 0xffffffffu;
    // Two passes of two dy each (dy = -8+4q+i0+i, i = 0, 1): the nine J rows
    // of a pass are each read from LDS once and used for both of its dy.
#pragma unroll 1
    for (int i0 = 0; i0 < 4; i0 += 2) {
        // acc[i][g]: four packed SADs of dx = -8+4g .. -5+4g; a8[i]: dx = +8
        uint64_t acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
        uint32_t a8[2] = {0, 0};
        const uint8_t* jb = sJ + (8 * by + 4 * q + i0) * kJW8 + 8 * bx;
        uint32_t off = 0;
#pragma unroll
        for (int u = 0; u < 9; ++u) {      // J row u pairs with block row j = u - i
            // the row's address passes through an empty asm that reads the
            // previous row's sum, so later rows are not hoisted into registers
            if (u > 0) asm volatile("" : "+v"(off) : "v"(a8[0]));
            const uint2 a = *reinterpret_cast<const uint2*>(jb + off);
            const uint2 b = *reinterpret_cast<const uint2*>(jb + off + 8);
            const uint2 c = *reinterpret_cast<const uint2*>(jb + off + 16);
            off += kJW8;
            const uint64_t w01 = pk64(a.x, a.y), w12 = pk64(a.y, b.x), w23 = pk64(b.x, b.y);
            const uint64_t w34 = pk64(b.y, c.x), w45 = pk64(c.x, c.y);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int j = u - i;
                if (j < 0 || j > 7) continue;
                acc[i][0] = __builtin_amdgcn_qsad_pk_u16_u8(w01, r0[j], acc[i][0]);
                acc[i][0] = __builtin_amdgcn_qsad_pk_u16_u8(w12, r1[j], acc[i][0]);
                acc[i][1] = __builtin_amdgcn_qsad_pk_u16_u8(w12, r0[j], acc[i][1]);
                acc[i][1] = __builtin_amdgcn_qsad_pk_u16_u8(w23, r1[j], acc[i][1]);
                acc[i][2] = __builtin_amdgcn_qsad_pk_u16_u8(w23, r0[j], acc[i][2]);
                acc[i][2] = __builtin_amdgcn_qsad_pk_u16_u8(w34, r1[j], acc[i][2]);
                acc[i][3] = __builtin_amdgcn_qsad_pk_u16_u8(w34, r0[j], acc[i][3]);
                acc[i][3] = __builtin_amdgcn_qsad_pk_u16_u8(w45, r1[j], acc[i][3]);
                a8[i] = __builtin_amdgcn_sad_u8(c.x, r0[j], a8[i]);
                a8[i] = __builtin_amdgcn_sad_u8(c.y, r1[j], a8[i]);
            }
        }
        // keys: the dx part of the code is a constant per candidate, the dy
        // part is added once per row (adding a constant keeps the row's argmin)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            uint32_t rb = (a8[i] << 16) + code_dx(8);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint32_t lo = (uint32_t)acc[i][g], hi = (uint32_t)(acc[i][g] >> 32);
                rb = min(rb, min((lo << 16) + code_dx(-8 + 4 * g), (lo & 0xffff0000u) + code_dx(-7 + 4 * g)));
                rb = min(rb, min((hi << 16) + code_dx(-6 + 4 * g), (hi & 0xffff0000u) + code_dx(-5 + 4 * g)));
            }
            best = min(best, rb + code_dy(-8 + 4 * q + i0 + i));
        }
    }
    // dy = +8 row, dx group q (dx = -8+4q .. -5+4q); lane q = 3 also dx = +8
    {
        uint64_t a4 = 0;
        uint32_t e8 = 0;
        const uint8_t* jr = sJ + (8 * by + 16) * kJW8 + 8 * bx + 4 * q;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e0 = *reinterpret_cast<const uint32_t*>(jr + j * kJW8);
            const uint32_t e1 = *reinterpret_cast<const uint32_t*>(jr + j * kJW8 + 4);
            const uint32_t e2 = *reinterpret_cast<const uint32_t*>(jr + j * kJW8 + 8);
            a4 = __builtin_amdgcn_qsad_pk_u16_u8(pk64(e0, e1), r0[j], a4);
            a4 = __builtin_amdgcn_qsad_pk_u16_u8(pk64(e1, e2), r1[j], a4);
            e8 = __builtin_amdgcn_sad_u8(e1, r0[j], e8);
            e8 = __builtin_amdgcn_sad_u8(e2, r1[j], e8);
        }
        const int dx0 = -8 + 4 * q;
        const uint32_t lo = (uint32_t)a4, hi = (uint32_t)(a4 >> 32);
        uint32_t rb = min((lo << 16) + code_dx(dx0), (lo & 0xffff0000u) + code_dx(dx0 + 1));
        rb = min(rb, min((hi << 16) + code_dx(dx0 + 2), (hi & 0xffff0000u) + code_dx(dx0 + 3)));
        if (q == 3) rb = min(rb, (e8 << 16) + code_dx(8));
        best = min(best, rb + code_dy(8));
    }
    return best;
}

// 10-bit search for one lane: returns the best key (SAD << 16) + code(dx, dy).
__device__ __forceinline__ uint32_t search16(const uint8_t* sI, const uint8_t* sJ, int bx, int by, int q) {
    // ref block: 8 rows x 4 dwords (2 samples each)
    uint32_t rf[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint4 v = *reinterpret_cast<const uint4*>(sI + ((8 * by + j) * 64 + 8 * bx) * 2);
        rf[j][0] = v.x; rf[j][1] = v.y; rf[j][2] = v.z; rf[j][3] = v.w;
    }
    uint32_t best = 0xffffffffu;
    constexpr int RB = kJW8 * 2;   // window row bytes
    const int ndy = (q == 3) ? 5 : 4;
    for (int i = 0; i < ndy; ++i) {
        const int dy = -8 + 4 * q + i;
        uint32_t acc[kCand];
#pragma unroll
        for (int k = 0; k < kCand; ++k) acc[k] = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // samples x0-8 .. x0+15 of window row 8 + 8*by + dy + j: 12 dwords
            const uint8_t* rowp = sJ + (8 * by + 8 + dy + j) * RB + 8 * bx * 2;
            uint32_t d[12];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint4 v = *reinterpret_cast<const uint4*>(rowp + 16 * k);
                d[4 * k] = v.x; d[4 * k + 1] = v.y; d[4 * k + 2] = v.z; d[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int dx = -8; dx <= 8; ++dx) {
                const int s = dx + 8;       // sample offset of the candidate in the window row
                uint32_t a = acc[dx + 8];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int so = s + 2 * m;   // sample index of the pair
                    uint32_t c;
                    if ((so & 1) == 0) c = d[so >> 1];
                    else c = __builtin_amdgcn_alignbyte(d[(so >> 1) + 1], d[so >> 1], 2);
                    a = __builtin_amdgcn_sad_u16(c, rf[j][m], a);
                }
                acc[dx + 8] = a;
            }
        }
        uint32_t rb = 0xffffffffu;
#pragma unroll
        for (int k = 0; k < kCand; ++k) rb = min(rb, (acc[k] << 16) + code_dx(k - kRadius));
        best = min(best, rb + code_dy(dy));
    }
    return best;
}

// Moments of one lane's two rows of the block against the warped J.
template <typename T>
__device__ __forceinline__ void moments(const uint8_t* sI, const uint8_t* sJ, int bx, int by, int q,
                                        int dx, int dy, int32_t m[5]) {
    for (int k = 0; k < 5; ++k) m[k] = 0;
    if constexpr (sizeof(T) == 1) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int j = 2 * q + jj;
            const uint2 xv = *reinterpret_cast<const uint2*>(sI + (8 * by + j) * 64 + 8 * bx);
            const int col = 8 * bx + 8 + dx;     // window byte column of the warped row
            const uint8_t* jr = sJ + (8 * by + 8 + dy + j) * kJW8 + (col & ~3);
            const uint32_t w0 = *reinterpret_cast<const uint32_t*>(jr);
            const uint32_t w1 = *reinterpret_cast<const uint32_t*>(jr + 4);
            const uint32_t w2 = ((col & 3) != 0) ? *reinterpret_cast<const uint32_t*>(jr + 8) : 0u;
            const int sh = col & 3;
            const uint32_t y0 = __builtin_amdgcn_alignbyte(w1, w0, sh);
            const uint32_t y1 = __builtin_amdgcn_alignbyte(w2, w1, sh);
            m[0] += (int32_t)(__builtin_amdgcn_sad_u8(xv.x, 0u, 0u) + __builtin_amdgcn_sad_u8(xv.y, 0u, 0u));
            m[1] += (int32_t)(__builtin_amdgcn_sad_u8(y0, 0u, 0u) + __builtin_amdgcn_sad_u8(y1, 0u, 0u));
            m[2] += (int32_t)__builtin_amdgcn_udot4(xv.y, xv.y, __builtin_amdgcn_udot4(xv.x, xv.x, 0u, false), false);
            m[3] += (int32_t)__builtin_amdgcn_udot4(y1, y1, __builtin_amdgcn_udot4(y0, y0, 0u, false), false);
            m[4] += (int32_t)__builtin_amdgcn_udot4(xv.y, y1, __builtin_amdgcn_udot4(xv.x, y0, 0u, false), false);
        }
    } else {
        constexpr int RB = kJW8 * 2;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int j = 2 * q + jj;
            const uint16_t* xr = reinterpret_cast<const uint16_t*>(sI + ((8 * by + j) * 64 + 8 * bx) * 2);
            const uint16_t* yr = reinterpret_cast<const uint16_t*>(sJ + (8 * by + 8 + dy + j) * RB) + 8 * bx + 8 + dx;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t x = xr[i], y = yr[i];
                m[0] += x; m[1] += y; m[2] += x * x; m[3] += y * y; m[4] += x * y;
            }
        }
    }
}

// Wavefront sum through the device library's reduction (DPP lane moves, no
// LDS crossbar round trips); every lane gets the total.
__device__ __forceinline__ int32_t wave_sum(int32_t v) {
    return __reduce_add_sync(~0ull, v);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Locate the task owning global tile `tile` in a prefix-sorted task list.
// SAD of one lane's two block rows at displacement (dx, dy) (debug output only).
template <typename T>
__device__ __forceinline__ int32_t rows_sad(const uint8_t* sI, const uint8_t* sJ, int bx, int by, int q,
                                            int dx, int dy) {
    constexpr int B = (int)sizeof(T);
    int32_t s = 0;
    for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * q + jj;
        const T* xr = reinterpret_cast<const T*>(sI + ((8 * by + j) * 64 + 8 * bx) * B);
        const T* yr = reinterpret_cast<const T*>(sJ + (8 * by + 8 + dy + j) * kJW8 * B) + 8 * bx + 8 + dx;
        for (int i = 0; i < 8; ++i) s += abs((int)xr[i] - (int)yr[i]);
    }
    return s;
}

template <typename T>
__device__ void me_tile(const TileJob& jb, int local, TilePartial* part_out, int8_t* mv_out, int32_t* sad_out,
                        uint8_t* sI, uint8_t* sJ, int64_t* red) {
    const PlaneRef I{jb.I, jb.w, jb.h, jb.pitch, jb.cos_I};
    const PlaneRef J{jb.J, jb.w, jb.h, jb.pitch, jb.cos_J};
    const int nbx = I.w / kBlock, nby = I.h / kBlock;
    const int tiles_x = jb.tiles_x;
    const int bx0 = (local % tiles_x) * kTBX, by0 = (local / tiles_x) * kTBY;
    stage_I<T>(I, bx0, by0, sI);
    stage_J<T>(J, bx0, by0, sJ);
    __syncthreads();
    const int tid = threadIdx.x;
    const int b = tid >> 2, q = tid & 3;
    const int bx = b & (kTBX - 1), by = b >> 3;
    const bool valid = (bx0 + bx < nbx) && (by0 + by < nby);
    int dx = 0, dy = 0;
    if (!(jb.flags & TF_ZERO_MV)) {
        uint32_t key = 0xffffffffu;
        if (valid) {
            if constexpr (sizeof(T) == 1) key = search8(sI, sJ, bx, by, q);
            else key = search16(sI, sJ, bx, by, q);
        }
        key = min(key, (uint32_t)__shfl_xor((int)key, 1, 64));
        key = min(key, (uint32_t)__shfl_xor((int)key, 2, 64));
        if (valid) {
            const uint32_t cell = (key & 0xffffu) % (uint32_t)(kCand * kCand);   // (dy+8)*17 + dx+8
            dx = (int)(cell % kCand) - kRadius;
            dy = (int)(cell / kCand) - kRadius;
        }
    }
    int32_t m[5] = {0, 0, 0, 0, 0};
    int32_t a = 0;
    if (valid) {
        moments<T>(sI, sJ, bx, by, q, dx, dy, m);
        if (q == 0) a = amm_fx(dx * dx + dy * dy);
    }
    const int blk = (by0 + by) * nbx + (bx0 + bx);
    if (sad_out) {
        int32_t s = valid ? rows_sad<T>(sI, sJ, bx, by, q, dx, dy) : 0;
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (valid && q == 0) sad_out[blk] = s;
    }
    if (mv_out && valid && q == 0) {
        mv_out[2 * blk] = (int8_t)dx;
        mv_out[2 * blk + 1] = (int8_t)dy;
    }
    // per-wave int32 sums are exact for 8- and 10-bit samples (16 blocks per wave)
    const int32_t w0 = wave_sum(m[0]), w1 = wave_sum(m[1]), w2 = wave_sum(m[2]);
    const int32_t w3 = wave_sum(m[3]), w4 = wave_sum(m[4]), w5 = wave_sum(a);
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
        red[wave * 6 + 0] = w0; red[wave * 6 + 1] = w1; red[wave * 6 + 2] = w2;
        red[wave * 6 + 3] = w3; red[wave * 6 + 4] = w4; red[wave * 6 + 5] = w5;
    }
    __syncthreads();
    if (tid == 0) {
        TilePartial p;
        p.sx = red[0] + red[6] + red[12] + red[18];
        p.sy = red[1] + red[7] + red[13] + red[19];
        p.sxx = red[2] + red[8] + red[14] + red[20];
        p.syy = red[3] + red[9] + red[15] + red[21];
        p.sxy = red[4] + red[10] + red[16] + red[22];
        p.a = red[5] + red[11] + red[17] + red[23];
        *part_out = p;
    }
    __syncthreads();   // LDS is reused by the next tile
}

}  // namespace

// Persistent grid over the tiles of the consecutive-pair list (host-built) and
// the sparse list (built on the device by the previous step's decision kernel).
// One launch per sample width; tiles of the other width are skipped.
template <typename T>
// One launch walks one tile list: the consecutive pairs of a step (n_tiles
// known to the host), or, with cur set, the sparse pairs planned by the
// previous step's decisions (their tile count read from cur->sparse_tt).
__global__ void __launch_bounds__(kMEThreads, 2) k_me(const StreamDesc* __restrict__ sds,
                                                   const TileJob* __restrict__ jobs, int32_t n_jobs,
                                                   const int32_t* __restrict__ map, int32_t n_tiles,
                                                   const DeviceCursors* __restrict__ cur, int32_t par_prev,
                                                   TilePartial* __restrict__ partials, int8_t* dbg_mv,
                                                   int32_t* dbg_sad, unsigned long long* __restrict__ clear_tt) {
    // clear this step's planning counter before the decision kernel adds to it
    if (clear_tt && blockIdx.x == 0 && threadIdx.x == 0) *clear_tt = 0ull;
    __shared__ __attribute__((aligned(16))) uint8_t sI[64 * 64 * sizeof(T)];
    __shared__ __attribute__((aligned(16))) uint8_t sJ[kJRows * kJW8 * sizeof(T)];
    __shared__ int64_t red[4 * 6];
    const bool sparse = cur != nullptr;
    // the sparse pairs precede the step's decisions on the critical path;
    // their waves issue before those of the next step's consecutive pairs
    if (sparse) __builtin_amdgcn_s_setprio(2);
    const int total = sparse ? tt_tiles(cur->sparse_tt[par_prev].v) : n_tiles;
    // Workgroups are dispatched round-robin over the XCDs, each with its own
    // L2: workgroup b runs on XCD b % kXcd.  Each XCD walks one contiguous
    // slice of the tile list, so neighbouring tiles of a pair (which share
    // cache lines of I and of the J halo) are fetched into the same L2.
    int lo = 0, hi = total, first = blockIdx.x, stride = gridDim.x;
    if (gridDim.x >= kXcd) {
        const int groups = gridDim.x / kXcd;      // the host launches a multiple of kXcd
        const int x = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
        if (j >= groups) return;
        const int per = (total + kXcd - 1) / kXcd;
        lo = x * per;
        hi = min(total, lo + per);
        first = lo + j;
        stride = groups;
    }
    // A tile's job: map entry, then the job (the next tile's map entry is
    // loaded one iteration ahead).  The consecutive pairs' jobs are built by
    // this step's pyramid kernel, the sparse pairs' by the previous step's
    // decision kernel.
    int idx_next = first < hi ? map[first] : 0;
    for (int tile = first; tile < hi; tile += stride) {
        const int idx = idx_next;
        const int nt = tile + stride;
        if (nt < hi) idx_next = map[nt];
        if (idx < 0 || idx >= n_jobs) continue;   // never expected; keeps reads in bounds
        const TileJob& jb = jobs[idx];
        const int local = tile - jb.tile_prefix;
        if (jb.bits != (sizeof(T) == 1 ? 8 : 10)) continue;
        if (sparse) {
            const StreamDesc& sd = sds[jb.sid];
            if (!sd.active || sd.epoch != jb.epoch) continue;   // stream closed since planning
        }
        const bool dbg = (jb.flags & TF_DEBUG) != 0;
        me_tile<T>(jb, local, partials + tile, dbg ? dbg_mv : jb.mv, dbg ? dbg_sad : nullptr, sI, sJ, red);
    }
}

// One wave per pair task: sum its tile partials and finish it.
__global__ void __launch_bounds__(256) k_finish(const StreamDesc* __restrict__ sds,
                                                const PairTask* __restrict__ consec, int32_t n_consec,
                                                int32_t consec_tiles, const PairTask* __restrict__ sparse,
                                                const DeviceCursors* __restrict__ cur,
                                                const TilePartial* __restrict__ partials,
                                                PairResult* __restrict__ results, DecideParams dp,
                                                int64_t* dbg_ints, double* dbg_dbl, int32_t par_prev,
                                                DeviceCursors* __restrict__ cur_w) {
    const int lane = threadIdx.x & 63;
    const int total = n_consec + (cur ? tt_tasks(cur->sparse_tt[par_prev].v) : 0);
    // clear this step's planning counter before the decision kernel adds to it
    if (cur_w && blockIdx.x == 0 && threadIdx.x == 0) cur_w->sparse_tt[par_prev ^ 1].v = 0ull;
    for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < total; t += gridDim.x * 4) {
        const bool is_consec = t < n_consec;
        const PairTask& tk = is_consec ? consec[t] : sparse[t - n_consec];
        if (!sds[tk.sid].active || sds[tk.sid].epoch != tk.epoch) continue;
        const int base = (is_consec ? 0 : consec_tiles) + tk.tile_prefix;
        int64_t s[6] = {0, 0, 0, 0, 0, 0};
        for (int i = lane; i < tk.tiles; i += 64) {
            const TilePartial& p = partials[base + i];
            s[0] += p.sx; s[1] += p.sy; s[2] += p.sxx; s[3] += p.syy; s[4] += p.sxy; s[5] += p.a;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = wave_sum64(s[k]);
        if (lane != 0) continue;
        const StreamDesc& sd = sds[tk.sid];
        const PlaneRef P = plane_of(sd, tk.ref, tk.ref_field, tk.level);
        const int64_t B = (int64_t)(P.w / kBlock) * (P.h / kBlock);
        const int64_t n = 64 * B;
        double f[4];
        finish_pair(s[0], s[1], s[2], s[3], s[4], n, s[5], B, dp.a0, f);
        if (tk.flags & TF_DEBUG) {
            if (dbg_ints) {
                dbg_ints[0] = s[0]; dbg_ints[1] = s[1]; dbg_ints[2] = s[2]; dbg_ints[3] = s[3];
                dbg_ints[4] = s[4]; dbg_ints[5] = n; dbg_ints[6] = s[5]; dbg_ints[7] = B;
                dbg_ints[8] = s[5] < (int64_t)dp.a_static_fx * B ? 1 : 0;
            }
            if (dbg_dbl) { dbg_dbl[0] = f[0]; dbg_dbl[1] = f[1]; dbg_dbl[2] = f[2]; dbg_dbl[3] = f[3]; }
        }
        if (is_consec) {
            FrameInfo& fi = sd.info[tk.ref % sd.rs];
            fi.ncc = f[0]; fi.swr = f[1]; fi.amm = f[2]; fi.act = f[3];
            for (int k = 0; k < 5; ++k) fi.mom[k] = s[k];
            fi.n_pix = n;
            fi.amm_num = s[5];
            fi.n_blocks = (int32_t)B;
            fi.flags |= VSA_F_HAS_PAIR | (s[5] < (int64_t)dp.a_static_fx * B ? VSA_F_STATIC : 0);
        } else if (tk.result >= 0) {
            PairResult& r = results[(int64_t)tk.sid * kResSlots + tk.result];
            r.act = f[3];
            r.swr = f[1];
        }
    }
}

// The finishing arithmetic alone on n tuples (bitwise check against the host).
__global__ void k_finish_debug(const int64_t* __restrict__ ints, int64_t n, double a0, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t* v = ints + 8 * i;
    double f[4];
    finish_pair(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], a0, f);
    out[4 * i] = f[0]; out[4 * i + 1] = f[1]; out[4 * i + 2] = f[2]; out[4 * i + 3] = f[3];
}

hipError_t launch_me(int bits, const StreamDesc* sds, const TileJob* jobs, int32_t n_jobs, const int32_t* map,
                     int32_t n_tiles, const DeviceCursors* cur, int32_t par_prev, bool clear_next, TilePartial* partials,
                     int8_t* dbg_mv, int32_t* dbg_sad, int grid, hipStream_t s, LaunchTiming tm) {
    if (grid <= 0) return hipSuccess;
    // the sparse launch of a step clears the planning counter the step's
    // decision kernel adds to (the other parity)
    unsigned long long* clear_tt =
        (cur && clear_next) ? const_cast<unsigned long long*>(&cur->sparse_tt[par_prev ^ 1].v) : nullptr;
    if (bits == 8) {
        if (tm.any())
            hipExtLaunchKernelGGL(k_me<uint8_t>, dim3(grid), dim3(kMEThreads), 0, s, tm.start, tm.stop, 0, sds,
                                  jobs, n_jobs, map, n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad, clear_tt);
        else
            hipLaunchKernelGGL(k_me<uint8_t>, dim3(grid), dim3(kMEThreads), 0, s, sds, jobs, n_jobs, map, n_tiles,
                               cur, par_prev, partials, dbg_mv, dbg_sad, clear_tt);
    } else {
        if (tm.any())
            hipExtLaunchKernelGGL(k_me<uint16_t>, dim3(grid), dim3(kMEThreads), 0, s, tm.start, tm.stop, 0, sds,
                                  jobs, n_jobs, map, n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad, clear_tt);
        else
            hipLaunchKernelGGL(k_me<uint16_t>, dim3(grid), dim3(kMEThreads), 0, s, sds, jobs, n_jobs, map, n_tiles,
                               cur, par_prev, partials, dbg_mv, dbg_sad, clear_tt);
    }
    return hipGetLastError();
}

hipError_t launch_finish(const StreamDesc* sds, const PairTask* consec, int32_t n_consec,
                         int32_t consec_tiles, const PairTask* sparse, DeviceCursors* cur,
                         const TilePartial* partials, PairResult* results, const DecideParams& dp,
                         int64_t* dbg_ints, double* dbg_dbl, int grid, int32_t par_prev, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(grid), dim3(256), 0, s, sds, consec, n_consec, consec_tiles, sparse,
                       cur, partials, results, dp, dbg_ints, dbg_dbl, par_prev, cur);
    return hipGetLastError();
}

hipError_t launch_finish_debug(const int64_t* ints, int64_t n, double a0, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_finish_debug, dim3((unsigned)grid), dim3(256), 0, s, ints, n, a0, out);
    return hipGetLastError();
}

}  // namespace vsa
