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
// pixels of I); a persistent grid walks the tile list.  The tile of I and its
// (64+16) x (64+16) search window of J are staged in LDS once (clamped at the
// plane edges), so every candidate is read from LDS.  Four lanes share a
// block: lane q searches dy in [-8+4q, -5+4q] over all dx and one quarter of
// the dy = +8 row.  8-bit: v_qsad_pk_u16_u8 gives the SADs of four
// consecutive dx from one aligned 8-byte window (dx groups -8, -4, 0, +4),
// v_sad_u8 covers dx = +8, so no byte alignment is ever needed in the search
// loop; each J row a lane needs is read from LDS once for two of its dy.  The
// 8-bit walk double-buffers the tiles in LDS: each thread loads its share of
// the next tile into registers while the current one is searched, with one
// barrier per tile.  10-bit: v_sad_u16 on pairs of samples with a 2-byte
// realignment for odd dx.  Each candidate's key is (SAD << 16) + code(dx, dy),
// where the code is strictly increasing in the candidate order (|d|^2, dy, dx)
// and below 2^16, so the minimum key is the unique argmin; the code is
// arithmetic, no table is read.  The epilogue reads the warped block from the
// same LDS window and forms int32 moments per lane, reduced per tile to int64.
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

// Key of the candidate whose 16-bit SAD sits in the low (SEL_LO) or high
// (SEL_HI) half of a packed accumulator: the SAD in the key's upper half, the
// tie-break code in its lower half, one byte permute (v_perm_b32) each.
constexpr uint32_t kSelLo = 0x05040100u;
constexpr uint32_t kSelHi = 0x07060100u;
__device__ __forceinline__ uint32_t key_of(uint32_t acc, uint32_t code, uint32_t sel) {
    return __builtin_amdgcn_perm(acc, code, sel);
}

// 8-bit search for one lane: returns the best key (SAD << 16) + code(dx, dy).
// two passes of two dy each, every J row of a pass read from LDS once and
// used for both dy; keys formed once per candidate with a byte permute and
// reduced with three-input minima.  Row u+1 of a pass is read before row u is
// searched; an empty asm after each row takes the row's sums and the row
// offset as in-out operands, so the compiler can neither defer the row's work
// past it nor hoist the loads of row u+2 above it (two J rows live at most).
__device__ __forceinline__ uint32_t search8p(const uint8_t* sI, const uint8_t* sJ, int bx, int by, int q) {
    uint32_t r0[8], r1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint2 v = *reinterpret_cast<const uint2*>(sI + (8 * by + j) * 64 + 8 * bx);
        r0[j] = v.x;
        r1[j] = v.y;
    }
    uint32_t best = 0xffffffffu;
#pragma unroll 1
    for (int i0 = 0; i0 < 4; i0 += 2) {
        // acc[i][g]: four packed SADs of dx = -8+4g .. -5+4g; a8[i]: dx = +8
        uint64_t acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
        uint32_t a8[2] = {0, 0};
        const uint8_t* jb = sJ + (8 * by + 4 * q + i0) * kJW8 + 8 * bx;
        uint32_t off = 0;
        uint2 na = *reinterpret_cast<const uint2*>(jb);
        uint2 nb = *reinterpret_cast<const uint2*>(jb + 8);
        uint2 nc = *reinterpret_cast<const uint2*>(jb + 16);
#pragma unroll
        for (int u = 0; u < 9; ++u) {      // J row u pairs with block row j = u - i
            const uint2 a = na, b = nb, c = nc;
            off += kJW8;
            if (u < 8) {
                na = *reinterpret_cast<const uint2*>(jb + off);
                nb = *reinterpret_cast<const uint2*>(jb + off + 8);
                nc = *reinterpret_cast<const uint2*>(jb + off + 16);
            }
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
                asm volatile("" : "+v"(acc[i][0]), "+v"(acc[i][1]), "+v"(acc[i][2]), "+v"(acc[i][3]),
                             "+v"(a8[i]), "+v"(off));
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            uint32_t rb = key_of(a8[i], code_dx(8), kSelLo);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint32_t lo = (uint32_t)acc[i][g], hi = (uint32_t)(acc[i][g] >> 32);
                rb = min(rb, min(key_of(lo, code_dx(-8 + 4 * g), kSelLo), key_of(lo, code_dx(-7 + 4 * g), kSelHi)));
                rb = min(rb, min(key_of(hi, code_dx(-6 + 4 * g), kSelLo), key_of(hi, code_dx(-5 + 4 * g), kSelHi)));
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
        uint32_t rb = min(key_of(lo, code_dx(dx0), kSelLo), key_of(lo, code_dx(dx0 + 1), kSelHi));
        rb = min(rb, min(key_of(hi, code_dx(dx0 + 2), kSelLo), key_of(hi, code_dx(dx0 + 3), kSelHi)));
        if (q == 3) rb = min(rb, key_of(e8, code_dx(8), kSelLo));
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
            if constexpr (sizeof(T) == 1) key = search8p(sI, sJ, bx, by, q);
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

// ---- 8-bit tiles: prefetched into registers, double-buffered in LDS -------

// One tile of 8 x 8 blocks, resolved from its job (uniform across the
// workgroup).
struct Tile8 {
    const uint8_t* I;
    const uint8_t* J;
    int8_t* mv;
    int w, h, pitch, cos_I, cos_J;
    int bx0, by0, flags;
};

// A thread's share of staging one tile: its 16-byte chunk of the I tile and
// up to four 8-byte chunks of the 80 x 80 J window (and, for a co-sited
// lower field, the same chunks one row higher).  Thread t holds J chunks
// i = t + 256 k (i < 800): window row i / 10, byte column 8 (i % 10), LDS
// offset 8 i; and I chunk t: row t / 4, byte column 16 (t % 4), LDS offset
// 16 t.
struct Stage8 {
    uint4 i0, i1;
    uint2 j0[4], j1[4];
};

constexpr int kJChunks8 = kJRows * (kJW8 / 8);   // 800

// Loads and stores through global-address-space pointers: the planes' and
// tiles' addresses come out of the jobs as generic pointers, and generic
// (flat) accesses count against the LDS wait counter too, so the search's
// first wait for an LDS read would also wait for the prefetched tile.
template <typename V>
__device__ __forceinline__ V gload(const uint8_t* p) {
    return *(const __attribute__((address_space(1))) V*)p;
}
template <typename V>
__device__ __forceinline__ void gstore(void* p, V v) {
    *(__attribute__((address_space(1))) V*)p = v;
}
__device__ __forceinline__ void store_partial(TilePartial* dst, const TilePartial& p) {
    int64_t* d = reinterpret_cast<int64_t*>(dst);
    gstore<int64_t>(d + 0, p.sx); gstore<int64_t>(d + 1, p.sy); gstore<int64_t>(d + 2, p.sxx);
    gstore<int64_t>(d + 3, p.syy); gstore<int64_t>(d + 4, p.sxy); gstore<int64_t>(d + 5, p.a);
}
__device__ __forceinline__ uint2 gload2(const uint8_t* p) {
    const uint64_t v = gload<uint64_t>(p);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}
__device__ __forceinline__ uint4 gload4(const uint8_t* p) {
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 v = gload<u64x2>(p);
    return make_uint4((uint32_t)v.x, (uint32_t)(v.x >> 32), (uint32_t)v.y, (uint32_t)(v.y >> 32));
}

// How a J chunk (8 bytes from byte column gx of the window row) is staged:
// whole within the plane, entirely left or right of it (every byte is the
// edge sample, one byte is loaded), or across the edge of a plane whose width
// is not a multiple of 8 (bytes loaded one by one when stored).
enum : int { JC_IN = 0, JC_LEFT = 1, JC_RIGHT = 2, JC_PART = 3 };
__device__ __forceinline__ int jclass(int gx, int w) {
    if (gx >= 0 && gx + 8 <= w) return JC_IN;
    if (gx + 8 <= 0) return JC_LEFT;
    if (gx >= w) return JC_RIGHT;
    return JC_PART;
}

__device__ __forceinline__ bool resolve8(const StreamDesc* __restrict__ sds, const TileJob* __restrict__ jobs,
                                         int n_jobs, int idx, int tile, bool sparse, int8_t* dbg_mv, Tile8& T) {
    if (idx < 0 || idx >= n_jobs) return false;   // never expected; keeps reads in bounds
    const TileJob& jb = jobs[idx];
    if (jb.bits != 8 || (jb.flags & (TF_HIER | TF_FLOW))) return false;
    if (sparse) {
        const StreamDesc& sd = sds[jb.sid];
        if (!sd.active || sd.epoch != jb.epoch) return false;   // stream closed since planning
    }
    const int local = tile - jb.tile_prefix;
    T.I = jb.I; T.J = jb.J;
    T.w = jb.w; T.h = jb.h; T.pitch = jb.pitch;
    T.cos_I = jb.cos_I; T.cos_J = jb.cos_J;
    T.bx0 = (local % jb.tiles_x) * kTBX;
    T.by0 = (local / jb.tiles_x) * kTBY;
    T.flags = jb.flags;
    T.mv = (jb.flags & TF_DEBUG) ? dbg_mv : jb.mv;
    return true;
}

// Global loads of a thread's chunks (no wait: they land while the previous
// tile is searched).  Window rows past the plane are clamped; the column
// class of a chunk is uniform over most tiles (inner columns all whole).
__device__ __forceinline__ void stage8_load(const Tile8& T, Stage8& S) {
    const int tid = threadIdx.x;
    {
        const int gy = min(8 * T.by0 + (tid >> 2), T.h - 1);
        const uint32_t o = (uint32_t)gy * (uint32_t)T.pitch + 8 * T.bx0 + 16 * (tid & 3);
        S.i0 = gload4(T.I + o);
        if (T.cos_I) S.i1 = gload4(T.I + (o - (gy > 0 ? T.pitch : 0)));
    }
    const int x0 = 8 * T.bx0 - 8, y0 = 8 * T.by0 - 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = tid + kMEThreads * k;
        if (k == 3 && i >= kJChunks8) break;
        const int r = i / (kJW8 / 8);
        const int gx = x0 + 8 * (i - r * (kJW8 / 8));
        const int gy = clampi(y0 + r, 0, T.h - 1);
        const uint32_t ro = (uint32_t)gy * (uint32_t)T.pitch;
        const uint32_t rp = gy > 0 ? ro - T.pitch : ro;
        const int cls = jclass(gx, T.w);
        if (cls == JC_IN) {
            S.j0[k] = gload2(T.J + ro + gx);
            if (T.cos_J) S.j1[k] = gload2(T.J + rp + gx);
        } else if (cls != JC_PART) {
            const uint32_t e = cls == JC_LEFT ? 0u : (uint32_t)(T.w - 1);
            S.j0[k].x = gload<uint8_t>(T.J + ro + e);
            if (T.cos_J) S.j1[k].x = gload<uint8_t>(T.J + rp + e);
        }
    }
}

__device__ __forceinline__ void stage8_store(const Tile8& T, const Stage8& S, uint8_t* sI, uint8_t* sJ) {
    const int tid = threadIdx.x;
    {
        uint4 v = S.i0;
        if (T.cos_I) v = cosite_vec<uint8_t, uint4>(v, S.i1, T.cos_I);
        reinterpret_cast<uint4*>(sI)[tid] = v;
    }
    const int x0 = 8 * T.bx0 - 8, y0 = 8 * T.by0 - 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = tid + kMEThreads * k;
        if (k == 3 && i >= kJChunks8) break;
        const int r = i / (kJW8 / 8);
        const int gx = x0 + 8 * (i - r * (kJW8 / 8));
        const int cls = jclass(gx, T.w);
        uint2 v = S.j0[k], w = S.j1[k];
        if (cls == JC_LEFT || cls == JC_RIGHT) {
            v.x = v.y = (v.x & 0xffu) * 0x01010101u;
            w.x = w.y = (w.x & 0xffu) * 0x01010101u;
        } else if (cls == JC_PART) {
            const int gy = clampi(y0 + r, 0, T.h - 1);
            const uint8_t* row = T.J + (uint32_t)gy * (uint32_t)T.pitch;
            const uint8_t* prv = T.J + (uint32_t)(gy > 0 ? gy - 1 : 0) * (uint32_t)T.pitch;
            union { uint8_t t[8]; uint2 u; } a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int x = clampi(gx + e, 0, T.w - 1);
                a.t[e] = gload<uint8_t>(row + x);
                b.t[e] = T.cos_J ? gload<uint8_t>(prv + x) : (uint8_t)0;
            }
            v = a.u;
            w = b.u;
        }
        if (T.cos_J) v = cosite_vec<uint8_t, uint2>(v, w, T.cos_J);
        reinterpret_cast<uint2*>(sJ)[i] = v;
    }
}

// The persistent walk over tiles lo..hi-1 (first, first+stride, ...) of one
// 8-bit launch.  Tile k+1's chunks are loaded into registers while tile k is
// searched and are written to the other LDS buffer at the top of the next
// iteration, so one barrier per tile separates the writes of a buffer from
// its reads (a buffer is rewritten two tiles later, after every thread has
// passed the barrier in between).  The four waves' moment sums of a tile go
// to a double-buffered LDS slot and are added by thread 0 after that barrier.
__device__ void me_walk8(const StreamDesc* __restrict__ sds, const TileJob* __restrict__ jobs, int n_jobs,
                         const int32_t* __restrict__ map, int hi, int first, int stride, bool sparse,
                         TilePartial* __restrict__ partials, int8_t* dbg_mv, int32_t* dbg_sad) {
    __shared__ __attribute__((aligned(16))) uint8_t sI[2][64 * 64];
    __shared__ __attribute__((aligned(16))) uint8_t sJ[2][kJRows * kJW8];
    __shared__ int32_t red[2][4 * 6];
    const int tid = threadIdx.x;
    const int b = tid >> 2, q = tid & 3;
    const int bx = b & (kTBX - 1), by = b >> 3;
    const int wave = tid >> 6;
    Stage8 S;
    // the job index of the tile whose chunks sit in S (re-resolved from the
    // job, which the scalar cache still holds, when they are stored), and the
    // map entry of the tile after it
    int idx_cur = first < hi ? map[first] : -1;
    int idx_nn = (first + stride < hi) ? map[first + stride] : -1;
    if (first < hi) {
        Tile8 t0;
        if (resolve8(sds, jobs, n_jobs, idx_cur, first, sparse, dbg_mv, t0)) stage8_load(t0, S);
    }
    int buf = 0;
    int pending = -1;           // tile whose wave sums wait in red[buf ^ 1]
    // Its motion vector (lane q = 0 of a valid block), stored after the next
    // barrier rather than at the end of the tile: a store still in flight at
    // the top of the next iteration would hold up the wait for that tile's
    // prefetched loads.
    int8_t* mv_dst = nullptr;
    int mv_blk = 0;
    uint32_t mv_val = 0;
    for (int tile = first; tile < hi; tile += stride) {
        Tile8 cur;
        const bool cur_ok = resolve8(sds, jobs, n_jobs, idx_cur, tile, sparse, dbg_mv, cur);
        if (cur_ok) stage8_store(cur, S, sI[buf], sJ[buf]);
        __syncthreads();
        // the next tile's loads go out first; the previous tile's results
        // are stored after them (neither waits for the other)
        const int nt = tile + stride;
        if (nt < hi) {
            idx_cur = idx_nn;
            idx_nn = (nt + stride < hi) ? map[nt + stride] : -1;
            Tile8 n;
            if (resolve8(sds, jobs, n_jobs, idx_cur, nt, sparse, dbg_mv, n)) stage8_load(n, S);
        }
        if (pending >= 0 && tid == 0) {
            const int32_t* rd = red[buf ^ 1];
            TilePartial p;
            p.sx = (int64_t)rd[0] + rd[6] + rd[12] + rd[18];
            p.sy = (int64_t)rd[1] + rd[7] + rd[13] + rd[19];
            p.sxx = (int64_t)rd[2] + rd[8] + rd[14] + rd[20];
            p.syy = (int64_t)rd[3] + rd[9] + rd[15] + rd[21];
            p.sxy = (int64_t)rd[4] + rd[10] + rd[16] + rd[22];
            p.a = (int64_t)rd[5] + rd[11] + rd[17] + rd[23];
            store_partial(partials + pending, p);
        }
        if (mv_dst) {
            gstore<uint8_t>(mv_dst + 2 * mv_blk, (uint8_t)(mv_val & 0xffu));
            gstore<uint8_t>(mv_dst + 2 * mv_blk + 1, (uint8_t)(mv_val >> 8));
        }
        mv_dst = nullptr;
        pending = -1;
        if (cur_ok) {
            const uint8_t* cI = sI[buf];
            const uint8_t* cJ = sJ[buf];
            const int nbx = cur.w / kBlock, nby = cur.h / kBlock;
            const bool valid = (cur.bx0 + bx < nbx) && (cur.by0 + by < nby);
            int dx = 0, dy = 0;
            if (!(cur.flags & TF_ZERO_MV)) {
                uint32_t key = valid ? search8p(cI, cJ, bx, by, q) : 0xffffffffu;
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
                moments<uint8_t>(cI, cJ, bx, by, q, dx, dy, m);
                if (q == 0) a = amm_fx(dx * dx + dy * dy);
            }
            const int blk = (cur.by0 + by) * nbx + (cur.bx0 + bx);
            if ((cur.flags & TF_DEBUG) && dbg_sad) {
                int32_t sd_ = valid ? rows_sad<uint8_t>(cI, cJ, bx, by, q, dx, dy) : 0;
                sd_ += __shfl_xor(sd_, 1, 64);
                sd_ += __shfl_xor(sd_, 2, 64);
                if (valid && q == 0) dbg_sad[blk] = sd_;
            }
            if (cur.mv && valid && q == 0) {
                mv_dst = cur.mv;
                mv_blk = blk;
                mv_val = (uint32_t)(dx & 0xff) | ((uint32_t)(dy & 0xff) << 8);
            }
            // per-wave int32 sums are exact for 8-bit samples (16 blocks per wave)
            const int32_t w0 = wave_sum(m[0]), w1 = wave_sum(m[1]), w2 = wave_sum(m[2]);
            const int32_t w3 = wave_sum(m[3]), w4 = wave_sum(m[4]), w5 = wave_sum(a);
            if ((tid & 63) == 0) {
                int32_t* rd = red[buf] + wave * 6;
                rd[0] = w0; rd[1] = w1; rd[2] = w2; rd[3] = w3; rd[4] = w4; rd[5] = w5;
            }
            pending = tile;
        }
        buf ^= 1;
    }
    __syncthreads();
    if (mv_dst) {
        gstore<uint8_t>(mv_dst + 2 * mv_blk, (uint8_t)(mv_val & 0xffu));
        gstore<uint8_t>(mv_dst + 2 * mv_blk + 1, (uint8_t)(mv_val >> 8));
    }
    if (pending >= 0 && tid == 0) {
        const int32_t* rd = red[buf ^ 1];
        TilePartial p;
        p.sx = (int64_t)rd[0] + rd[6] + rd[12] + rd[18];
        p.sy = (int64_t)rd[1] + rd[7] + rd[13] + rd[19];
        p.sxx = (int64_t)rd[2] + rd[8] + rd[14] + rd[20];
        p.syy = (int64_t)rd[3] + rd[9] + rd[15] + rd[21];
        p.sxy = (int64_t)rd[4] + rd[10] + rd[16] + rd[22];
        p.a = (int64_t)rd[5] + rd[11] + rd[17] + rd[23];
        store_partial(partials + pending, p);
    }
}


// ---- coarse-to-fine motion field (frame pairs of streams with search = 1) --
//
// A tile is 16 x 16 blocks (128 x 128 samples) of I.  First the coarse I tile
// (64 x 64, 8 x 8 coarse blocks) and the coarse J window (80 x 80 around it,
// clamped to the coarse plane) are formed in LDS straight from the fine
// planes in memory (2 x 2 box averages, the pyramid's own step), laid out as
// the full search stages its tiles, so the coarse vectors come from the full
// search's lane code.  Then, for each half of the tile (8 block rows), the
// fine I rows and a fine J window (rows -17 .., columns fx0-24 .., clamped to
// the plane) are staged and two lanes take each fine block: prediction =
// twice its coarse block's vector (when that coarse block is whole), the best
// of prediction + e, e in [-1, 1]^2, and the warped moments, each lane over
// four of the block's rows.
constexpr int kHT = kHTB * kBlock;       // 128 samples per tile side
constexpr int kHHR = kHT / 2;            // fine rows per half tile
constexpr int kHOX = 24;                 // window column of fine column fx0
constexpr int kHOY = 17;                 // window row of the half's first fine row
constexpr int kHJW = 176;                // window row length (samples)
constexpr int kHJH = kHHR + 2 * kHOY;    // 98 window rows per half
static_assert(kHOX % 8 == 0 && kHJW % 8 == 0, "window chunks are 8 samples");
// a refinement or moment reads up to column 8*15 + kHOX + 17 + 11 and row
// 8*7 + 7 + 17 + kHOY of the half's window
static_assert(8 * 15 + kHOX + 16 + 11 < kHJW && 8 * 7 + 7 + 17 + kHOY < kHJH, "window too small");

template <typename T>
struct HierLds {
    uint8_t cI[64 * 64 * sizeof(T)];
    uint8_t cJ[kJRows * kJW8 * sizeof(T)];
    uint8_t fI[kHHR * kHT * sizeof(T)];
    uint8_t fJ[kHJH * kHJW * sizeof(T)];
    int32_t cmv[64];                      // coarse vector per coarse block: dx & 0xff | (dy & 0xff) << 8
    int64_t red[4 * 6];
};

// 2 x 2 box averages (rounding half up) of four coarse samples from two fine
// rows of eight samples (8 bytes, or 16 bytes of 16-bit samples):
// v_dot4_u32_u8 / v_dot2_u32_u16 against a mask add the two samples of a
// column pair of each row onto the rounding constant; the four results are
// packed into the coarse row's four samples.
typedef unsigned short hpk_us2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t box_pair8(uint32_t a, uint32_t b, uint32_t m) {
    return __builtin_amdgcn_udot4(a, m, __builtin_amdgcn_udot4(b, m, 2u, false), false) >> 2;
}
__device__ __forceinline__ uint32_t box_pair16(uint32_t a, uint32_t b) {
    const hpk_us2 one = {1, 1};
    return __builtin_amdgcn_udot2(__builtin_bit_cast(hpk_us2, a), one,
                                  __builtin_amdgcn_udot2(__builtin_bit_cast(hpk_us2, b), one, 2u, false), false) >> 2;
}
template <typename T>
__device__ __forceinline__ void box4_global(const uint8_t* r0, const uint8_t* r1, T* dst) {
    if constexpr (sizeof(T) == 1) {
        const uint2 a = gload2(r0), b = gload2(r1);
        const uint32_t s0 = box_pair8(a.x, b.x, 0x00000101u), s1 = box_pair8(a.x, b.x, 0x01010000u);
        const uint32_t s2 = box_pair8(a.y, b.y, 0x00000101u), s3 = box_pair8(a.y, b.y, 0x01010000u);
        *reinterpret_cast<uint32_t*>(dst) = s0 | (s1 << 8) | (s2 << 16) | (s3 << 24);
    } else {
        const uint4 a = gload4(r0), b = gload4(r1);
        const uint32_t s0 = box_pair16(a.x, b.x), s1 = box_pair16(a.y, b.y);
        const uint32_t s2 = box_pair16(a.z, b.z), s3 = box_pair16(a.w, b.w);
        *reinterpret_cast<uint2*>(dst) = make_uint2(s0 | (s1 << 16), s2 | (s3 << 16));
    }
}

// The coarse tile and window, from the fine planes in memory.  Coarse I
// items past the row pitch are not read (their blocks are not whole); coarse
// rows past the plane read its last fine rows.  Window items whose columns
// reach past the coarse plane's edge clamp each column on its own.
template <typename T>
__device__ void hier_coarse(const TileJob& jb, int fx0, int fy0, HierLds<T>& S) {
    constexpr int B = (int)sizeof(T);
    const int tid = threadIdx.x;
    T* cI = reinterpret_cast<T*>(S.cI);
    T* cJ = reinterpret_cast<T*>(S.cJ);
    if (jb.cI) {
        // the coarse tile and window straight from the stored coarser level
        // (a quarter of the bytes).  Coarse I items past its row pitch or its
        // rows belong to no whole coarse block and are not read; window rows
        // and columns clamp to the coarse plane (w / 2 x h / 2) as above.
        const int wc = jb.w / 2, hc = jb.h / 2;
        const int ccx = fx0 / 2, ccy = fy0 / 2;
        for (int i = tid; i < 64 * 16; i += kMEThreads) {
            const int y = i >> 4, x = 4 * (i & 15);
            const int cx = ccx + x, cy = ccy + y;
            T* dst = cI + y * 64 + x;
            if (cx >= jb.cpitch || cy >= hc) {
                if constexpr (B == 1) *reinterpret_cast<uint32_t*>(dst) = 0u;
                else *reinterpret_cast<uint2*>(dst) = make_uint2(0u, 0u);
                continue;
            }
            const uint8_t* src = jb.cI + ((int64_t)cy * jb.cpitch + cx) * B;
            if constexpr (B == 1) *reinterpret_cast<uint32_t*>(dst) = gload<uint32_t>(src);
            else *reinterpret_cast<uint2*>(dst) = gload2(src);
        }
        const int cx0 = ccx - 8, cy0 = ccy - 8;
        constexpr int G = kJW8 / 4;
        for (int i = tid; i < kJRows * G; i += kMEThreads) {
            const int r = i / G, c = 4 * (i - (i / G) * G);
            const int cy = clampi(cy0 + r, 0, hc - 1);
            const uint8_t* row = jb.cJ + (int64_t)cy * jb.cpitch * B;
            T* dst = cJ + r * kJW8 + c;
            if (cx0 + c >= 0 && cx0 + c + 3 <= wc - 1) {
                if constexpr (B == 1) *reinterpret_cast<uint32_t*>(dst) = gload<uint32_t>(row + (cx0 + c));
                else *reinterpret_cast<uint2*>(dst) = gload2(row + 2 * (cx0 + c));
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) dst[k] = gload<T>(row + clampi(cx0 + c + k, 0, wc - 1) * B);
            }
        }
        return;
    }
    for (int i = tid; i < 64 * 16; i += kMEThreads) {
        const int y = i >> 4, x = 4 * (i & 15);
        const int gx = fx0 + 2 * x;
        if (gx >= jb.pitch) {
            if constexpr (B == 1) *reinterpret_cast<uint32_t*>(cI + y * 64 + x) = 0u;
            else *reinterpret_cast<uint2*>(cI + y * 64 + x) = make_uint2(0u, 0u);
            continue;
        }
        const int g0 = min(fy0 + 2 * y, jb.h - 1), g1 = min(fy0 + 2 * y + 1, jb.h - 1);
        box4_global<T>(jb.I + ((int64_t)g0 * jb.pitch + gx) * B, jb.I + ((int64_t)g1 * jb.pitch + gx) * B,
                       cI + y * 64 + x);
    }
    const int wc = jb.w / 2, hc = jb.h / 2;
    const int cx0 = fx0 / 2 - 8, cy0 = fy0 / 2 - 8;
    constexpr int G = kJW8 / 4;                      // items per window row
    for (int i = tid; i < kJRows * G; i += kMEThreads) {
        const int r = i / G, c = 4 * (i - (i / G) * G);
        const int cy = clampi(cy0 + r, 0, hc - 1);
        const uint8_t* r0 = jb.J + (int64_t)(2 * cy) * jb.pitch * B;
        const uint8_t* r1 = r0 + (int64_t)jb.pitch * B;
        T* dst = cJ + r * kJW8 + c;
        if (cx0 + c >= 0 && cx0 + c + 3 <= wc - 1) {
            box4_global<T>(r0 + 2 * (cx0 + c) * B, r1 + 2 * (cx0 + c) * B, dst);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int f = 2 * clampi(cx0 + c + k, 0, wc - 1);
                dst[k] = (T)(((int)gload<T>(r0 + f * B) + gload<T>(r0 + (f + 1) * B) + gload<T>(r1 + f * B) +
                              gload<T>(r1 + (f + 1) * B) + 2) >> 2);
            }
        }
    }
}

// Fine I rows fy0 + 64 hh .. +64 and the half's J window (rows from
// fy0 + 64 hh - kHOY, columns from fx0 - kHOX), clamped to the plane; I
// chunks past the row pitch are not read.
template <typename T>
__device__ void hier_stage_half(const TileJob& jb, int fx0, int fy0, int hh, HierLds<T>& S) {
    constexpr int B = (int)sizeof(T);
    const int tid = threadIdx.x;
    const int ry = fy0 + kHHR * hh;
    constexpr int ICH = kHT * B / 16;
    for (int i = tid; i < kHHR * ICH; i += kMEThreads) {
        const int r = i / ICH, c = i - (i / ICH) * ICH;
        const int gy = min(ry + r, jb.h - 1);
        const int gx = fx0 + c * (16 / B);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gx < jb.pitch) v = gload4(jb.I + ((int64_t)gy * jb.pitch + gx) * B);
        reinterpret_cast<uint4*>(S.fI)[i] = v;
    }
    constexpr int JCH = kHJW / 8;
    const int x0 = fx0 - kHOX, y0 = ry - kHOY;
    for (int i = tid; i < kHJH * JCH; i += kMEThreads) {
        const int r = i / JCH, c = i - (i / JCH) * JCH;
        const int gy = clampi(y0 + r, 0, jb.h - 1);
        const int gx = x0 + 8 * c;
        const uint8_t* row = jb.J + (int64_t)gy * jb.pitch * B;
        T* dst = reinterpret_cast<T*>(S.fJ) + r * kHJW + 8 * c;
        if (gx >= 0 && gx + 8 <= jb.w) {
            if constexpr (B == 1) *reinterpret_cast<uint2*>(dst) = gload2(row + gx);
            else *reinterpret_cast<uint4*>(dst) = gload4(row + 2 * gx);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[k] = gload<T>(row + clampi(gx + k, 0, jb.w - 1) * B);
        }
    }
}

// Key of refinement candidate e: SAD << 16 | code, the code increasing in
// (|e|^2, ey, ex).
__device__ __forceinline__ uint32_t hier_key(uint32_t sad, int ex, int ey) {
    return (sad << 16) | (uint32_t)(((ex * ex + ey * ey) * 3 + ey + 1) * 3 + ex + 1);
}

// 8-bit partial refinement of half-tile block (bx, by) over its rows j0 ..
// j0+3, around prediction (px, py) (both even): v_qsad_pk_u16_u8 over the
// two dx groups q-4 .. q-1 and q .. q+3, q = px rounded down to a multiple
// of 4, which hold the candidates px-1 .. px+1; each J row is read once for
// the three ey.  acc[ey+1][group]: four packed 16-bit partial SADs.
__device__ __forceinline__ void hier_refine8(const uint8_t* fI, const uint8_t* fJ, int bx, int by, int j0, int px,
                                             int py, uint64_t (&acc)[3][2]) {
    uint32_t r0[4], r1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint2 v = *reinterpret_cast<const uint2*>(fI + (8 * by + j0 + j) * kHT + 8 * bx);
        r0[j] = v.x;
        r1[j] = v.y;
    }
    const int q4 = px & ~3;
    const uint8_t* jb = fJ + (8 * by + j0 + py + kHOY - 1) * kHJW + (8 * bx + kHOX + q4 - 4);
#pragma unroll
    for (int e = 0; e < 3; ++e) acc[e][0] = acc[e][1] = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {            // J row u holds row j = u - 1 - ey of the lane's four
        const uint32_t* wp = reinterpret_cast<const uint32_t*>(jb + u * kHJW);
        const uint32_t w0 = wp[0], w1 = wp[1], w2 = wp[2], w3 = wp[3];
        const uint64_t w01 = pk64(w0, w1), w12 = pk64(w1, w2), w23 = pk64(w2, w3);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int j = u - e;
            if (j < 0 || j > 3) continue;
            acc[e][0] = __builtin_amdgcn_qsad_pk_u16_u8(w01, r0[j], acc[e][0]);
            acc[e][0] = __builtin_amdgcn_qsad_pk_u16_u8(w12, r1[j], acc[e][0]);
            acc[e][1] = __builtin_amdgcn_qsad_pk_u16_u8(w12, r0[j], acc[e][1]);
            acc[e][1] = __builtin_amdgcn_qsad_pk_u16_u8(w23, r1[j], acc[e][1]);
        }
    }
}

// The key of the best candidate from the summed packed SADs.
__device__ __forceinline__ uint32_t hier_best8(const uint64_t (&acc)[3][2], int px) {
    const bool h2 = (px & 3) != 0;           // px = q4 or q4 + 2
    uint32_t best = 0xffffffffu;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const uint64_t a0 = acc[e][0], a1 = acc[e][1];
        const uint32_t sm = h2 ? (uint32_t)(a1 >> 16) & 0xffffu : (uint32_t)(a0 >> 48);
        const uint32_t s0 = h2 ? (uint32_t)(a1 >> 32) & 0xffffu : (uint32_t)a1 & 0xffffu;
        const uint32_t sp = h2 ? (uint32_t)(a1 >> 48) : (uint32_t)(a1 >> 16) & 0xffffu;
        best = min(best, min(hier_key(sm, -1, e - 1), min(hier_key(s0, 0, e - 1), hier_key(sp, 1, e - 1))));
    }
    return best;
}

// 10-bit partial refinement over rows j0 .. j0+3: sad[ey+1][ex+1].
__device__ __forceinline__ void hier_refine16(const uint8_t* fI, const uint8_t* fJ, int bx, int by, int j0, int px,
                                              int py, uint32_t (&sad)[3][3]) {
    const uint16_t* I = reinterpret_cast<const uint16_t*>(fI) + (8 * by + j0) * kHT + 8 * bx;
    const uint16_t* J =
        reinterpret_cast<const uint16_t*>(fJ) + (8 * by + j0 + py + kHOY - 1) * kHJW + (8 * bx + px + kHOX - 1);
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int f = 0; f < 3; ++f) sad[e][f] = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        int jr[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) jr[k] = J[u * kHJW + k];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int j = u - e;
            if (j < 0 || j > 3) continue;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int x = I[j * kHT + i];
#pragma unroll
                for (int f = 0; f < 3; ++f) sad[e][f] += (uint32_t)abs(x - jr[i + f]);
            }
        }
    }
}

// Moments of rows j0 .. j0+3 of half-tile block (bx, by) against J warped by (dx, dy).
template <typename T>
__device__ __forceinline__ void hier_moments(const uint8_t* fI, const uint8_t* fJ, int bx, int by, int j0, int dx,
                                             int dy, int32_t s[5]) {
    if constexpr (sizeof(T) == 1) {
        const int col = 8 * bx + kHOX + dx;
#pragma unroll
        for (int j = j0; j < j0 + 4; ++j) {
            const uint2 xv = *reinterpret_cast<const uint2*>(fI + (8 * by + j) * kHT + 8 * bx);
            const uint8_t* jr = fJ + (8 * by + j + dy + kHOY) * kHJW + (col & ~3);
            const uint32_t w0 = *reinterpret_cast<const uint32_t*>(jr);
            const uint32_t w1 = *reinterpret_cast<const uint32_t*>(jr + 4);
            const uint32_t w2 = *reinterpret_cast<const uint32_t*>(jr + 8);
            const int sh = col & 3;
            const uint32_t y0 = __builtin_amdgcn_alignbyte(w1, w0, sh);
            const uint32_t y1 = __builtin_amdgcn_alignbyte(w2, w1, sh);
            s[0] += (int32_t)(__builtin_amdgcn_sad_u8(xv.x, 0u, 0u) + __builtin_amdgcn_sad_u8(xv.y, 0u, 0u));
            s[1] += (int32_t)(__builtin_amdgcn_sad_u8(y0, 0u, 0u) + __builtin_amdgcn_sad_u8(y1, 0u, 0u));
            s[2] += (int32_t)__builtin_amdgcn_udot4(xv.y, xv.y, __builtin_amdgcn_udot4(xv.x, xv.x, 0u, false), false);
            s[3] += (int32_t)__builtin_amdgcn_udot4(y1, y1, __builtin_amdgcn_udot4(y0, y0, 0u, false), false);
            s[4] += (int32_t)__builtin_amdgcn_udot4(xv.y, y1, __builtin_amdgcn_udot4(xv.x, y0, 0u, false), false);
        }
    } else {
        const uint16_t* I = reinterpret_cast<const uint16_t*>(fI) + (8 * by + j0) * kHT + 8 * bx;
        const uint16_t* J =
            reinterpret_cast<const uint16_t*>(fJ) + (8 * by + j0 + dy + kHOY) * kHJW + (8 * bx + dx + kHOX);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t x = I[j * kHT + i], y = J[j * kHJW + i];
                s[0] += x; s[1] += y; s[2] += x * x; s[3] += y * y; s[4] += x * y;
            }
    }
}

// The fine blocks of half hh of a staged tile: two lanes per block (lane pair
// 2 k, 2 k + 1: rows 0-3 and 4-7), refinement around the coarse prediction,
// the vector and SAD out, moments and A into the lane's sums.
template <typename T>
__device__ __forceinline__ void hier_half(const TileJob& jb, HierLds<T>& S, int tx, int ty, int hh, bool coarse,
                                          bool zero, int8_t* mv_out, int32_t* sad_out, int32_t s[5], int32_t& a) {
    const int tid = threadIdx.x;
    const int nbx = jb.w / kBlock, nby = jb.h / kBlock;
    const int nbxc = (jb.w / 2) / kBlock, nbyc = (jb.h / 2) / kBlock;
    const int hl = tid & 1, k = tid >> 1;
    const int bx = k & (kHTB - 1), byh = k / kHTB;    // block column, block row within the half
    const int by = kHTB / 2 * hh + byh;               // block row within the tile
    const bool valid = (kHTB * tx + bx < nbx) && (kHTB * ty + by < nby);
    int dx = 0, dy = 0;
    uint32_t best = 0;
    if (!zero) {
        int px = 0, py = 0;
        if (coarse && kHTB / 2 * tx + (bx >> 1) < nbxc && kHTB / 2 * ty + (by >> 1) < nbyc) {
            const int v = S.cmv[(by >> 1) * 8 + (bx >> 1)];
            px = 2 * (int)(int8_t)(v & 0xff);
            py = 2 * (int)(int8_t)((v >> 8) & 0xff);
        }
        // both lanes of a pair run the same code; an invalid block's lanes
        // read inside the window and their result is not used
        if constexpr (sizeof(T) == 1) {
            uint64_t acc[3][2];
            hier_refine8(S.fI, S.fJ, bx, byh, 4 * hl, px, py, acc);
#pragma unroll
            for (int e = 0; e < 3; ++e)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const uint64_t o = (uint64_t)__shfl_xor((long long)acc[e][g], 1, 64);
                    acc[e][g] += o;   // 16-bit lanes: each sum stays below 64 * 255
                }
            best = hier_best8(acc, px);
        } else {
            uint32_t sd[3][3];
            hier_refine16(S.fI, S.fJ, bx, byh, 4 * hl, px, py, sd);
            best = 0xffffffffu;
#pragma unroll
            for (int e = 0; e < 3; ++e)
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const uint32_t t = sd[e][f] + (uint32_t)__shfl_xor((int)sd[e][f], 1, 64);
                    best = min(best, hier_key(t, f - 1, e - 1));
                }
        }
        const int code = (int)(best & 0xffffu) % 9;      // (ey+1)*3 + ex+1
        dx = px + code % 3 - 1;
        dy = py + code / 3 - 1;
    }
    if (valid) {
        hier_moments<T>(S.fI, S.fJ, bx, byh, 4 * hl, dx, dy, s);
        if (hl == 0) a += amm_fx(dx * dx + dy * dy);
    }
    const int blk = (kHTB * ty + by) * nbx + (kHTB * tx + bx);
    if (valid && hl == 0 && mv_out) {
        mv_out[2 * blk] = (int8_t)dx;
        mv_out[2 * blk + 1] = (int8_t)dy;
    }
    if (sad_out) {
        int32_t sv = 0;
        if (zero) {
            const T* I = reinterpret_cast<const T*>(S.fI) + (8 * byh + 4 * hl) * kHT + 8 * bx;
            const T* J = reinterpret_cast<const T*>(S.fJ) + (8 * byh + 4 * hl + kHOY) * kHJW + (8 * bx + kHOX);
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 8; ++i) sv += abs((int)I[j * kHT + i] - (int)J[j * kHJW + i]);
            sv += __shfl_xor(sv, 1, 64);
        } else {
            sv = (int32_t)(best >> 16);
        }
        if (valid && hl == 0) sad_out[blk] = sv;
    }
}

// Coarse vectors of the tile's coarse blocks (four lanes per coarse block, as
// in a full-search tile) into S.cmv.
template <typename T>
__device__ __forceinline__ void hier_coarse_search(const TileJob& jb, HierLds<T>& S, int tx, int ty) {
    const int tid = threadIdx.x;
    const int nbxc = (jb.w / 2) / kBlock, nbyc = (jb.h / 2) / kBlock;
    const int b = tid >> 2, q = tid & 3;
    const int cbx = b & 7, cby = b >> 3;
    const bool cvalid = (8 * tx + cbx < nbxc) && (8 * ty + cby < nbyc);
    uint32_t key = 0xffffffffu;
    if (cvalid) {
        if constexpr (sizeof(T) == 1) key = search8p(S.cI, S.cJ, cbx, cby, q);
        else key = search16(S.cI, S.cJ, cbx, cby, q);
    }
    key = min(key, (uint32_t)__shfl_xor((int)key, 1, 64));
    key = min(key, (uint32_t)__shfl_xor((int)key, 2, 64));
    if (q == 0) {
        int v = 0;
        if (cvalid) {
            const uint32_t cell = (key & 0xffffu) % (uint32_t)(kCand * kCand);   // (dy+8)*17 + dx+8
            const int dx = (int)(cell % kCand) - kRadius, dy = (int)(cell / kCand) - kRadius;
            v = (dx & 0xff) | ((dy & 0xff) << 8);
        }
        S.cmv[b] = v;
    }
}

// One coarse-to-fine tile: the vectors of its fine blocks, their moments and
// A, one partial per tile.
__device__ __forceinline__ const uint8_t* uniform_ptr(const uint8_t* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<const uint8_t*>(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ void me_tile_hier(const TileJob& job, int local, TilePartial* part_out, int8_t* mv_out, int32_t* sad_out,
                             HierLds<T>& S) {
    // the job is the same for the whole workgroup: its fields in scalar
    // registers, so that the staging addresses are a scalar base plus a
    // 32-bit lane offset
    TileJob jb = job;
    jb.I = uniform_ptr(job.I);
    jb.J = uniform_ptr(job.J);
    jb.cI = uniform_ptr(job.cI);
    jb.cJ = uniform_ptr(job.cJ);
    jb.cpitch = __builtin_amdgcn_readfirstlane(job.cpitch);
    jb.w = __builtin_amdgcn_readfirstlane(job.w);
    jb.h = __builtin_amdgcn_readfirstlane(job.h);
    jb.pitch = __builtin_amdgcn_readfirstlane(job.pitch);
    jb.tiles_x = __builtin_amdgcn_readfirstlane(job.tiles_x);
    jb.flags = __builtin_amdgcn_readfirstlane(job.flags);
    const int tid = threadIdx.x;
    const int tx = local % jb.tiles_x, ty = local / jb.tiles_x;
    const int fx0 = tx * kHT, fy0 = ty * kHT;
    const int nbxc = (jb.w / 2) / kBlock, nbyc = (jb.h / 2) / kBlock;
    const bool zero = (jb.flags & TF_ZERO_MV) != 0;
    // the coarse stage runs when the coarse plane has a whole block (else every
    // prediction is (0, 0))
    const bool coarse = !zero && nbxc > 0 && nbyc > 0;
    int32_t s[5] = {0, 0, 0, 0, 0};
    int32_t a = 0;
    if (coarse) {
        hier_coarse<T>(jb, fx0, fy0, S);
        __syncthreads();
        hier_coarse_search<T>(jb, S, tx, ty);
    }
    for (int hh = 0; hh < 2; ++hh) {
        __syncthreads();                               // the previous half's (or the coarse stage's) reads are done
        hier_stage_half<T>(jb, fx0, fy0, hh, S);
        __syncthreads();
        hier_half<T>(jb, S, tx, ty, hh, coarse, zero, mv_out, sad_out, s, a);
    }
    // per lane: half of each of two blocks; int64 wave sums (10-bit squares)
    const int wave = tid >> 6;
    int64_t w[6];
#pragma unroll
    for (int q = 0; q < 5; ++q) w[q] = wave_sum64((int64_t)s[q]);
    w[5] = wave_sum64((int64_t)a);
    if ((tid & 63) == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) S.red[wave * 6 + q] = w[q];
    __syncthreads();
    if (tid == 0) {
        TilePartial p;
        p.sx = S.red[0] + S.red[6] + S.red[12] + S.red[18];
        p.sy = S.red[1] + S.red[7] + S.red[13] + S.red[19];
        p.sxx = S.red[2] + S.red[8] + S.red[14] + S.red[20];
        p.syy = S.red[3] + S.red[9] + S.red[15] + S.red[21];
        p.sxy = S.red[4] + S.red[10] + S.red[16] + S.red[22];
        p.a = S.red[5] + S.red[11] + S.red[17] + S.red[23];
        store_partial(part_out, p);
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
    const bool sparse = cur != nullptr;
    // the sparse pairs precede the step's decisions on the critical path;
    // their waves issue before those of the next step's consecutive pairs,
    // which in turn issue before the pyramid's (HBM-bound, it has slack)
    if (sparse) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(1);
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
    // A tile's job: map entry, then the job.  The consecutive pairs' jobs are
    // built by this step's pyramid kernel, the sparse pairs' by the previous
    // step's decision kernel.
    if constexpr (sizeof(T) == 1) {
        me_walk8(sds, jobs, n_jobs, map, hi, first, stride, sparse, partials, dbg_mv, dbg_sad);
    } else {
        // 10-bit: one LDS buffer; the next tile's map entry is loaded one
        // iteration ahead
        __shared__ __attribute__((aligned(16))) uint8_t sI[64 * 64 * sizeof(T)];
        __shared__ __attribute__((aligned(16))) uint8_t sJ[kJRows * kJW8 * sizeof(T)];
        __shared__ int64_t red[4 * 6];
        int idx_next = first < hi ? map[first] : 0;
        for (int tile = first; tile < hi; tile += stride) {
            const int idx = idx_next;
            const int nt = tile + stride;
            if (nt < hi) idx_next = map[nt];
            if (idx < 0 || idx >= n_jobs) continue;   // never expected; keeps reads in bounds
            const TileJob& jb = jobs[idx];
            const int local = tile - jb.tile_prefix;
            if (jb.bits != 10 || (jb.flags & (TF_HIER | TF_FLOW))) continue;
            if (sparse) {
                const StreamDesc& sd = sds[jb.sid];
                if (!sd.active || sd.epoch != jb.epoch) continue;   // stream closed since planning
            }
            const bool dbg = (jb.flags & TF_DEBUG) != 0;
            me_tile<T>(jb, local, partials + tile, dbg ? dbg_mv : jb.mv, dbg ? dbg_sad : nullptr, sI, sJ, red);
        }
    }
}

// Persistent grid over the coarse-to-fine tiles of a tile list (the same
// lists, maps and jobs as k_me; tiles of full-search pairs and of the other
// sample width are skipped).  One workgroup of 256 lanes per 16 x 16-block
// tile, the XCD slicing of k_me.
template <typename T>
__global__ void __launch_bounds__(kMEThreads) k_me_hier(const StreamDesc* __restrict__ sds,
                                                        const TileJob* __restrict__ jobs, int32_t n_jobs,
                                                        const int32_t* __restrict__ map, int32_t n_tiles,
                                                        const DeviceCursors* __restrict__ cur, int32_t par_prev,
                                                        TilePartial* __restrict__ partials, int8_t* dbg_mv,
                                                        int32_t* dbg_sad) {
    __shared__ __attribute__((aligned(16))) HierLds<T> S;
    const bool sparse = cur != nullptr;
    if (sparse) __builtin_amdgcn_s_setprio(2);
    const int total = sparse ? tt_tiles(cur->sparse_tt[par_prev].v) : n_tiles;
    int lo = 0, hi = total, first = blockIdx.x, stride = gridDim.x;
    if (gridDim.x >= kXcd) {
        const int groups = gridDim.x / kXcd;
        const int x = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
        if (j >= groups) return;
        const int per = (total + kXcd - 1) / kXcd;
        lo = x * per;
        hi = min(total, lo + per);
        first = lo + j;
        stride = groups;
    }
    for (int tile = first; tile < hi; tile += stride) {
        const int idx = map[tile];
        if (idx < 0 || idx >= n_jobs) continue;   // never expected; keeps reads in bounds
        const TileJob& jb = jobs[idx];
        if (jb.bits != (sizeof(T) == 1 ? 8 : 10) || !(jb.flags & TF_HIER)) continue;
        if (sparse) {
            const StreamDesc& sd = sds[jb.sid];
            if (!sd.active || sd.epoch != jb.epoch) continue;   // stream closed since planning
        }
        const bool dbg = (jb.flags & TF_DEBUG) != 0;
        me_tile_hier<T>(jb, tile - jb.tile_prefix, partials + tile, dbg ? dbg_mv : jb.mv, dbg ? dbg_sad : nullptr,
                        S);
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
        if (sds[tk.sid].search == 2) {
            // the dense flow: the pair's tiles hold its row sums
            const StreamDesc& sd = sds[tk.sid];
            const PlaneRef P = plane_of(sd, tk.ref, tk.ref_field, tk.level);
            const FlowFinish f =
                flow_finish(reinterpret_cast<const FlowRow*>(partials + base), P.w, P.h, dp.a0, dp.a_static_fx);
            if (lane != 0) continue;
            const int64_t n = (int64_t)P.w * P.h;
            if (tk.flags & TF_DEBUG) {
                if (dbg_ints) {
                    for (int k = 0; k < 9; ++k) dbg_ints[k] = 0;
                    dbg_ints[5] = n;
                    dbg_ints[8] = f.is_static ? 1 : 0;
                }
                if (dbg_dbl) { dbg_dbl[0] = f.ncc; dbg_dbl[1] = f.swr; dbg_dbl[2] = f.amm; dbg_dbl[3] = f.act; }
            }
            if (is_consec) {
                FrameInfo& fi = sd.info[tk.ref % sd.rs];
                fi.ncc = f.ncc; fi.swr = f.swr; fi.amm = f.amm; fi.act = f.act;
                for (int k = 0; k < 5; ++k) fi.mom[k] = 0;
                fi.n_pix = n;
                fi.amm_num = 0;
                fi.n_blocks = 0;
                fi.flags |= VSA_F_HAS_PAIR | (f.is_static ? VSA_F_STATIC : 0);
            } else if (tk.result >= 0) {
                PairResult& r = results[(int64_t)tk.sid * kResSlots + tk.result];
                r.act = f.act;
                r.swr = f.swr;
            }
            continue;
        }
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

// Workgroups of the motion-search kernel one compute unit holds at once (its
// registers and LDS decide); persistent grids are sized within it, since a
// workgroup that waits for room would start its share of tiles late.
int me_max_wgs_per_cu(int bits) {
    static int cached[2] = {0, 0};
    int& c = cached[bits == 8 ? 0 : 1];
    if (c == 0) {
        int n = 0;
        const hipError_t e = bits == 8
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_me<uint8_t>, kMEThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_me<uint16_t>, kMEThreads, 0);
        c = (e == hipSuccess && n > 0) ? n : 2;
    }
    return c;
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

int me_hier_max_wgs_per_cu(int bits) {
    static int cached[2] = {0, 0};
    int& c = cached[bits == 8 ? 0 : 1];
    if (c == 0) {
        int n = 0;
        const hipError_t e = bits == 8
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_me_hier<uint8_t>, kMEThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_me_hier<uint16_t>, kMEThreads, 0);
        c = (e == hipSuccess && n > 0) ? n : 1;
    }
    return c;
}

hipError_t launch_me_hier(int bits, const StreamDesc* sds, const TileJob* jobs, int32_t n_jobs, const int32_t* map,
                          int32_t n_tiles, const DeviceCursors* cur, int32_t par_prev, TilePartial* partials,
                          int8_t* dbg_mv, int32_t* dbg_sad, int grid, hipStream_t s, LaunchTiming tm) {
    if (grid <= 0) return hipSuccess;
    if (bits == 8) {
        if (tm.any())
            hipExtLaunchKernelGGL(k_me_hier<uint8_t>, dim3(grid), dim3(kMEThreads), 0, s, tm.start, tm.stop, 0, sds,
                                  jobs, n_jobs, map, n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad);
        else
            hipLaunchKernelGGL(k_me_hier<uint8_t>, dim3(grid), dim3(kMEThreads), 0, s, sds, jobs, n_jobs, map,
                               n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad);
    } else {
        if (tm.any())
            hipExtLaunchKernelGGL(k_me_hier<uint16_t>, dim3(grid), dim3(kMEThreads), 0, s, tm.start, tm.stop, 0, sds,
                                  jobs, n_jobs, map, n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad);
        else
            hipLaunchKernelGGL(k_me_hier<uint16_t>, dim3(grid), dim3(kMEThreads), 0, s, sds, jobs, n_jobs, map,
                               n_tiles, cur, par_prev, partials, dbg_mv, dbg_sad);
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
