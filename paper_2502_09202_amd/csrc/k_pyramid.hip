// k_pyramid.hip -- K1: luma pyramid and fields of every frame ingested in a step.
//
// Each frame level is the 2x2 box average of the level below, rounded half up
// and applied once per level (a trailing odd row/column is dropped); the upper
// field holds the even rows and the lower field the odd rows of the frame
// (Sec. III.C), reduced the same way to the field level Lf = max(0, L-1).
//
// One 256-thread workgroup covers a 64 x 16 tile of the working level L.
// Every thread reads a band of 2^L rows x 4*2^L columns of the luma plane with
// 16-byte loads (the plane is read exactly once), reduces it level by level in
// registers to 4 working-level pixels and 8 pixels of each field, and stores
// them.  The coarser levels L+1..L+4 used by the long-range deep-check pairs
// are reduced from the 64 x 16 tile held in LDS, so the full-resolution plane
// is never read again.  The kernel is HBM-bound: bytes moved per frame are the
// plane plus the levels written.
//
// The same pass counts the working-level pixels of each tile into an LDS
// histogram and writes it out, for the unary intensity measure of Sec. III.A;
// k_intensity (queued right after, one workgroup per frame) sums the tile
// histograms, stores the frame histogram in the ring slot and forms the mean,
// standard deviation and mean absolute deviation from exact integer sums
// (mean = S1/N, std = sqrt(N S2 - S1^2)/N, mad = sum h[v] |N v - S1| / N^2),
// each rounded once.  (A last-tile-of-the-frame reduction inside this kernel
// would need a device-scope release per workgroup, which writes back the
// XCD's L2 each time.)
#include "vsa_internal.h"

#include <algorithm>

namespace vsa {

namespace {

template <int N>
struct Row {
    int v[N];
};

template <int N>
__device__ __forceinline__ Row<N / 2> down2(const Row<N>& a, const Row<N>& b) {
    Row<N / 2> o;
#pragma unroll
    for (int i = 0; i < N / 2; ++i)
        o.v[i] = (a.v[2 * i] + a.v[2 * i + 1] + b.v[2 * i] + b.v[2 * i + 1] + 2) >> 2;
    return o;
}

// Load NC samples of one luma row starting at column x0 (zeros past the edge;
// such samples only feed outputs that are never stored).
template <typename T, int NC>
__device__ __forceinline__ void load_row(const uint8_t* rowp, int x0, int W, bool al16,
                                         Row<NC>& o) {
    const T* p = reinterpret_cast<const T*>(rowp) + x0;
    constexpr int BYTES = NC * (int)sizeof(T);
    if (x0 + NC <= W && al16 && BYTES % 16 == 0) {
        const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            const uint4 u = q[k];
            uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (sizeof(T) == 1) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) o.v[16 * k + 4 * m + b] = (w4[m] >> (8 * b)) & 0xff;
                } else {
                    o.v[8 * k + 2 * m] = w4[m] & 0xffff;
                    o.v[8 * k + 2 * m + 1] = w4[m] >> 16;
                }
            }
        }
    } else if (x0 + NC <= W && al16 && BYTES % 4 == 0) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
        for (int k = 0; k < BYTES / 4; ++k) {
            uint32_t w = q[k];
            if (sizeof(T) == 1) {
#pragma unroll
                for (int b = 0; b < 4; ++b) o.v[4 * k + b] = (w >> (8 * b)) & 0xff;
            } else {
                o.v[2 * k] = w & 0xffff;
                o.v[2 * k + 1] = w >> 16;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NC; ++i) o.v[i] = (x0 + i < W) ? (int)p[i] : 0;
    }
}

// Frame row at level l and field rows at level l-1 of a band of 2^l luma rows.
template <int NC, int l>
struct Band {
    Row<(NC >> l)> f;
    Row<(NC >> (l - 1))> u, d;
};

template <typename T, int NC, int l>
__device__ __forceinline__ void build_band(const uint8_t* src, int64_t pitch, int y0, int x0, int W,
                                           bool al16, Band<NC, l>& out) {
    if constexpr (l == 1) {
        Row<NC> a, b;
        load_row<T, NC>(src + (int64_t)y0 * pitch, x0, W, al16, a);
        load_row<T, NC>(src + (int64_t)(y0 + 1) * pitch, x0, W, al16, b);
        out.f = down2<NC>(a, b);
        out.u = a;
        out.d = b;
    } else {
        Band<NC, l - 1> top, bot;
        build_band<T, NC, l - 1>(src, pitch, y0, x0, W, al16, top);
        build_band<T, NC, l - 1>(src, pitch, y0 + (1 << (l - 1)), x0, W, al16, bot);
        out.f = down2<(NC >> (l - 1))>(top.f, bot.f);
        out.u = down2<(NC >> (l - 2))>(top.u, bot.u);
        out.d = down2<(NC >> (l - 2))>(top.d, bot.d);
    }
}

// Working levels 2 and 3: the 2x2 box sums straight from packed samples, with
// dot products against a mask (v_dot4_u32_u8 adds two bytes of a word,
// v_dot2_u32_u16 the two samples of a word; two rows accumulate onto the
// rounding constant 2), instead of unpacking every sample.  Same arithmetic
// as down2, level by level.  Words past the plane's width read as 0 (they
// only feed outputs that are never stored), as in load_row.
typedef unsigned short pk_us2 __attribute__((ext_vector_type(2)));

template <typename T> struct Pk;
template <> struct Pk<uint8_t> {
    static constexpr int E = 4;   // samples per 32-bit word
    static constexpr int C = 2;   // level-1 columns per word
    static __device__ __forceinline__ uint32_t box(uint32_t a, uint32_t b, int h) {
        const uint32_t m = h ? 0x01010000u : 0x00000101u;
        return __builtin_amdgcn_udot4(a, m, __builtin_amdgcn_udot4(b, m, 2u, false), false) >> 2;
    }
};
template <> struct Pk<uint16_t> {
    static constexpr int E = 2;
    static constexpr int C = 1;
    static __device__ __forceinline__ uint32_t box(uint32_t a, uint32_t b, int) {
        const pk_us2 one = {1, 1};
        return __builtin_amdgcn_udot2(__builtin_bit_cast(pk_us2, a), one,
                                      __builtin_amdgcn_udot2(__builtin_bit_cast(pk_us2, b), one, 2u, false),
                                      false) >> 2;
    }
};

// NW words of one row starting at sample x0.
template <typename T, int NW>
__device__ __forceinline__ void load_words(const uint8_t* rowp, int x0, int W, bool fast, uint32_t (&w)[NW]) {
    constexpr int E = Pk<T>::E;
    const T* p = reinterpret_cast<const T*>(rowp) + x0;
    if (fast) {
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) {
            const uint4 q = reinterpret_cast<const uint4*>(p)[k];
            w[4 * k] = q.x; w[4 * k + 1] = q.y; w[4 * k + 2] = q.z; w[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            uint32_t v = 0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (x0 + E * k + e < W) v |= (uint32_t)p[E * k + e] << ((32 / E) * e);
            w[k] = v;
        }
    }
}

// Level-1 column j of rows (a, b): word j / C, pair j % C.
template <typename T, int NW>
__device__ __forceinline__ int l1col(const uint32_t (&a)[NW], const uint32_t (&b)[NW], int j) {
    return (int)Pk<T>::box(a[j / Pk<T>::C], b[j / Pk<T>::C], j % Pk<T>::C);
}

// A band of 2^L rows x NC samples (L = 2: 16 = 4 x 4; L = 3: 16 = 2 x 8): the
// frame value(s) at level L and both fields at level L-1.
template <typename T, int L, int NC>
__device__ __forceinline__ void band_dot(const uint8_t* src, int64_t pitch, int y0, int x0, int W, bool al16,
                                         Row<(NC >> L)>& f, Row<(NC >> (L - 1))>& u, Row<(NC >> (L - 1))>& d) {
    constexpr int NW = NC / Pk<T>::E;
    const bool fast = al16 && x0 + NC <= W;
    if constexpr (L == 2) {
        uint32_t w0[NW], w1[NW], w2[NW], w3[NW];
        load_words<T, NW>(src + (int64_t)(y0 + 0) * pitch, x0, W, fast, w0);
        load_words<T, NW>(src + (int64_t)(y0 + 1) * pitch, x0, W, fast, w1);
        load_words<T, NW>(src + (int64_t)(y0 + 2) * pitch, x0, W, fast, w2);
        load_words<T, NW>(src + (int64_t)(y0 + 3) * pitch, x0, W, fast, w3);
#pragma unroll
        for (int i = 0; i < (NC >> 2); ++i) {   // level 1 of rows (0,1) and (2,3), then level 2
            const int a0 = l1col<T>(w0, w1, 2 * i), a1 = l1col<T>(w0, w1, 2 * i + 1);
            const int b0 = l1col<T>(w2, w3, 2 * i), b1 = l1col<T>(w2, w3, 2 * i + 1);
            f.v[i] = (a0 + a1 + b0 + b1 + 2) >> 2;
        }
#pragma unroll
        for (int j = 0; j < (NC >> 1); ++j) {   // fields at level 1: rows (0,2) and (1,3)
            u.v[j] = l1col<T>(w0, w2, j);
            d.v[j] = l1col<T>(w1, w3, j);
        }
    } else {
        static_assert(L == 3, "working levels 2 and 3");
        int l2[2][NC >> 2], uf[2][NC >> 1], df[2][NC >> 1];
#pragma unroll
        for (int h = 0; h < 2; ++h) {           // rows 4h .. 4h+3
            uint32_t w0[NW], w1[NW], w2[NW], w3[NW];
            load_words<T, NW>(src + (int64_t)(y0 + 4 * h + 0) * pitch, x0, W, fast, w0);
            load_words<T, NW>(src + (int64_t)(y0 + 4 * h + 1) * pitch, x0, W, fast, w1);
            load_words<T, NW>(src + (int64_t)(y0 + 4 * h + 2) * pitch, x0, W, fast, w2);
            load_words<T, NW>(src + (int64_t)(y0 + 4 * h + 3) * pitch, x0, W, fast, w3);
#pragma unroll
            for (int k = 0; k < (NC >> 2); ++k) {
                const int a0 = l1col<T>(w0, w1, 2 * k), a1 = l1col<T>(w0, w1, 2 * k + 1);
                const int b0 = l1col<T>(w2, w3, 2 * k), b1 = l1col<T>(w2, w3, 2 * k + 1);
                l2[h][k] = (a0 + a1 + b0 + b1 + 2) >> 2;
            }
#pragma unroll
            for (int j = 0; j < (NC >> 1); ++j) {   // fields at level 1: rows (4h, 4h+2), (4h+1, 4h+3)
                uf[h][j] = l1col<T>(w0, w2, j);
                df[h][j] = l1col<T>(w1, w3, j);
            }
        }
#pragma unroll
        for (int i = 0; i < (NC >> 3); ++i)
            f.v[i] = (l2[0][2 * i] + l2[0][2 * i + 1] + l2[1][2 * i] + l2[1][2 * i + 1] + 2) >> 2;
#pragma unroll
        for (int k = 0; k < (NC >> 2); ++k) {   // fields at level 2
            u.v[k] = (uf[0][2 * k] + uf[0][2 * k + 1] + uf[1][2 * k] + uf[1][2 * k + 1] + 2) >> 2;
            d.v[k] = (df[0][2 * k] + df[0][2 * k + 1] + df[1][2 * k] + df[1][2 * k + 1] + 2) >> 2;
        }
    }
}

template <typename T, int N>
__device__ __forceinline__ void store_row(uint8_t* dst, int x0, int w, const Row<N>& r) {
    T* p = reinterpret_cast<T*>(dst) + x0;
    if (x0 + N <= w) {
        if constexpr (sizeof(T) == 1 && N == 4) {
            *reinterpret_cast<uint32_t*>(p) =
                (uint32_t)r.v[0] | ((uint32_t)r.v[1] << 8) | ((uint32_t)r.v[2] << 16) | ((uint32_t)r.v[3] << 24);
            return;
        } else if constexpr (sizeof(T) == 1 && N == 8) {
            uint2 u;
            u.x = (uint32_t)r.v[0] | ((uint32_t)r.v[1] << 8) | ((uint32_t)r.v[2] << 16) | ((uint32_t)r.v[3] << 24);
            u.y = (uint32_t)r.v[4] | ((uint32_t)r.v[5] << 8) | ((uint32_t)r.v[6] << 16) | ((uint32_t)r.v[7] << 24);
            *reinterpret_cast<uint2*>(p) = u;
            return;
        } else if constexpr (sizeof(T) == 1 && N == 2) {
            *reinterpret_cast<uint16_t*>(p) = (uint16_t)(r.v[0] | (r.v[1] << 8));
            return;
        } else if constexpr (sizeof(T) == 2 && N == 2) {
            *reinterpret_cast<uint32_t*>(p) = (uint32_t)r.v[0] | ((uint32_t)r.v[1] << 16);
            return;
        } else if constexpr (sizeof(T) == 2 && N == 4) {
            uint2 u;
            u.x = (uint32_t)r.v[0] | ((uint32_t)r.v[1] << 16);
            u.y = (uint32_t)r.v[2] | ((uint32_t)r.v[3] << 16);
            *reinterpret_cast<uint2*>(p) = u;
            return;
        } else if constexpr (sizeof(T) == 2 && N == 8) {
            uint4 u;
            u.x = (uint32_t)r.v[0] | ((uint32_t)r.v[1] << 16);
            u.y = (uint32_t)r.v[2] | ((uint32_t)r.v[3] << 16);
            u.z = (uint32_t)r.v[4] | ((uint32_t)r.v[5] << 16);
            u.w = (uint32_t)r.v[6] | ((uint32_t)r.v[7] << 16);
            *reinterpret_cast<uint4*>(p) = u;
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (x0 + i < w) p[i] = (T)r.v[i];
}

__device__ __forceinline__ uint8_t* slot_base(const StreamDesc& sd, int frame) {
    return sd.ring + (int64_t)(frame % sd.rs) * sd.slot_bytes;
}

// Working-level columns per thread: 4 up to L = 2, fewer for larger L so that
// the per-thread band (2^L rows x CW 2^L columns) stays small in registers.
template <int L>
struct PyrShape {
    static constexpr int CW = L <= 2 ? 4 : (L == 3 ? 2 : 1);
    static constexpr int TW = 16 * CW;     // tile width (working-level pixels)
};

__host__ __device__ inline int pyr_cw(int L) { return L <= 2 ? 4 : (L == 3 ? 2 : 1); }

// Pyramid grid width (working-level columns) covering the level and the fields.
__host__ __device__ inline int pyr_grid_w(const StreamDesc& sd) {
    const int shift = sd.L - sd.Lf;          // 1 for L >= 1, 0 for L == 0
    const int gw = (sd.wf + (1 << shift) - 1) >> shift;
    return gw > sd.wl[0] ? gw : sd.wl[0];
}

template <typename T, int L>
__device__ void pyramid_tile(const StreamDesc& sd, const StepStream& ss, int tile, uint16_t* lds, uint32_t* hist) {
    constexpr int S = 1 << L;
    constexpr int CW = PyrShape<L>::CW;
    constexpr int TW = PyrShape<L>::TW;
    constexpr int NC = CW * S;
    const int tiles_x = div_up(pyr_grid_w(sd), TW);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int c = threadIdx.x & 15, r = threadIdx.x >> 4;
    const int X = tx * TW + CW * c;           // first working-level column of this thread
    const int YL = ty * kPyrTH + r;           // working-level row
    const uint8_t* src = reinterpret_cast<const uint8_t*>(ss.src);
    const int64_t pitch = ss.src_pitch;
    const bool al16 = ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)pitch) & 15) == 0;
    uint8_t* slot = slot_base(sd, ss.frame);
    const int wL = sd.wl[0], hL = sd.hl[0];

    Row<CW> fl;
    if (YL < hL) {
        if constexpr (L == 0) {
            Row<CW> a;
            load_row<T, CW>(src + (int64_t)YL * pitch, X, sd.W, al16, a);
            fl = a;
            // fields at level 0: even rows -> upper, odd rows -> lower
            const int fy = YL >> 1;
            if (fy < sd.hf) {
                uint8_t* dst = slot + ((YL & 1) ? sd.offD : sd.offU) + (int64_t)fy * sd.pf * (int64_t)sizeof(T);
                store_row<T, CW>(dst, X, sd.wf, a);
            }
        } else {
            Band<NC, L> b;
            if constexpr (L == 2 || L == 3) {
                band_dot<T, L, NC>(src, pitch, YL * S, X * S, sd.W, al16, b.f, b.u, b.d);
            } else {
                build_band<T, NC, L>(src, pitch, YL * S, X * S, sd.W, al16, b);
            }
            fl = b.f;
            if (YL < sd.hf) {
                const int64_t rowoff = (int64_t)YL * sd.pf * (int64_t)sizeof(T);
                store_row<T, 2 * CW>(slot + sd.offU + rowoff, 2 * X, sd.wf, b.u);
                store_row<T, 2 * CW>(slot + sd.offD + rowoff, 2 * X, sd.wf, b.d);
            }
        }
        store_row<T, CW>(slot + sd.off[0] + (int64_t)YL * sd.pl[0] * (int64_t)sizeof(T), X, wL, fl);
        if (hist && X < wL) {
            // a run of equal adjacent values is one atomic (fewer lanes of a
            // wave on one LDS address in smooth regions); a bin index is kept
            // below 2^bits even for samples outside the 10-bit range (which the
            // host refuses for planes it copies; a device plane is read as is)
            constexpr int kMaxBin = sizeof(T) == 1 ? 255 : 1023;
            int cur = fl.v[0];
            uint32_t cnt = 1;
#pragma unroll
            for (int i = 1; i < CW; ++i) {
                if (X + i >= wL) break;
                if (fl.v[i] == cur) {
                    ++cnt;
                } else {
                    atomicAdd(&hist[min(cur, kMaxBin)], cnt);
                    cur = fl.v[i];
                    cnt = 1;
                }
            }
            atomicAdd(&hist[min(cur, kMaxBin)], cnt);
        }
    } else {
#pragma unroll
        for (int i = 0; i < CW; ++i) fl.v[i] = 0;
    }
    if (sd.nlev <= 1) return;
    // coarser levels from the tile in LDS
#pragma unroll
    for (int i = 0; i < CW; ++i) lds[r * TW + CW * c + i] = (uint16_t)fl.v[i];
    __syncthreads();
    uint16_t* prev = lds;
    uint16_t* next = lds + kPyrTW * kPyrTH;
    int pw = TW, ph = kPyrTH;
    for (int d = 1; d < sd.nlev; ++d) {
        const int cw = pw >> 1, ch = ph >> 1;
        const int i = threadIdx.x;
        if (i < cw * ch) {
            const int x = i % cw, y = i / cw;
            const int v = (prev[(2 * y) * pw + 2 * x] + prev[(2 * y) * pw + 2 * x + 1] +
                           prev[(2 * y + 1) * pw + 2 * x] + prev[(2 * y + 1) * pw + 2 * x + 1] + 2) >> 2;
            next[y * cw + x] = (uint16_t)v;
            const int gx = tx * (TW >> d) + x, gy = ty * (kPyrTH >> d) + y;
            if (gx < sd.wl[d] && gy < sd.hl[d]) {
                T* dst = reinterpret_cast<T*>(slot + sd.off[d]) + (int64_t)gy * sd.pl[d] + gx;
                *dst = (T)v;
            }
        }
        __syncthreads();
        uint16_t* tmp = prev;
        prev = next;
        next = tmp;
        pw = cw;
        ph = ch;
    }
}

// After the tile's pixels are counted in `hist`: store the tile histogram
// (at most 64 x 16 pixels per tile: the counts fit 16 bits).
template <typename T>
__device__ void store_tile_hist(const StreamDesc& sd, int tile, const uint32_t* hist) {
    constexpr int NB = sizeof(T) == 1 ? 256 : 1024;
    __syncthreads();                               // every count of the tile is in
    uint16_t* th = sd.tileh + (int64_t)tile * NB;
    for (int v = threadIdx.x; v < NB; v += 256) th[v] = (uint16_t)hist[v];
}

__device__ __forceinline__ void init_frame_info(const StreamDesc& sd, const StepStream& ss) {
    FrameInfo& fi = sd.info[ss.frame % sd.rs];
    const double nan = __builtin_nan("");
    fi.frame = ss.frame;
    fi.pts = ss.pts;
    fi.flags = ss.frame == 0 ? (VSA_F_KEYFRAME | VSA_F_SHOT_START) : 0;
    fi.shot_id = -1;
    fi.boundary = 0;
    fi.boundary_k = 0;
    fi.ncc = fi.swr = fi.amm = fi.act = nan;
    for (int i = 0; i < 5; ++i) fi.mom[i] = 0;
    fi.n_pix = 0;
    fi.amm_num = 0;
    fi.n_blocks = 0;
    fi.field_mask = 0;
    fi.v[0] = fi.v[1] = fi.v[2] = nan;
    fi.h_mean = fi.h_std = fi.h_mad = nan;
}

}  // namespace

// Grid: one workgroup per pyramid tile over the ingesting streams of one
// (sample width, working level) group; each group is its own instantiation so
// that registers are sized for that shape only.
template <typename T, int L>
__global__ void __launch_bounds__(256, (sizeof(T) == 1 && L <= 2) ? 7 : 1) k_pyramid(const StreamDesc* __restrict__ sds,
                                                  const StepStream* __restrict__ steps,
                                                  const int32_t* __restrict__ k1_list, int32_t n_k1,
                                                  TileJob* __restrict__ cjobs, int32_t* __restrict__ cmap) {
    __shared__ uint16_t lds[2 * kPyrTW * kPyrTH];
    __shared__ uint32_t hist[sizeof(T) == 1 ? 256 : 1024];
    const int tile = blockIdx.x;
    // locate the stream: last list entry whose first tile is <= tile
    int lo = 0, hi = n_k1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (steps[k1_list[mid]].k1_prefix <= tile) lo = mid; else hi = mid - 1;
    }
    const StepStream& ss = steps[k1_list[lo]];
    const int local = tile - ss.k1_prefix;
    if (local < 0 || local >= ss.k1_tiles) return;
    const StreamDesc& sd = sds[ss.sid];
    if (local == 0) {
        if (threadIdx.x == 0) init_frame_info(sd, ss);
        // the motion-search job of this step's consecutive pair (frame-1 ->
        // frame) and the map from its tiles to that job
        if (cjobs && ss.has_frame && ss.consec_tiles > 0) {
            const int i = k1_list[lo];
            if (threadIdx.x == 0) {
                PairTask t;
                t.sid = ss.sid; t.kind = MK_CONSEC; t.ref = ss.frame - 1; t.oth = ss.frame;
                t.ref_field = t.oth_field = PL_FRAME; t.level = sd.L; t.result = -1;
                t.tiles = ss.consec_tiles; t.tile_prefix = ss.consec_prefix; t.flags = TF_MV_RING;
                t.epoch = sd.epoch;
                cjobs[i] = make_tile_job(sd, t, sd.mv + (int64_t)(t.ref % sd.rs) * sd.B_L * 2);
            }
            for (int k = threadIdx.x; k < ss.consec_tiles; k += 256) cmap[ss.consec_prefix + k] = i;
        }
    }
    const bool unary = sd.tileh != nullptr;
    if (unary) {
        for (int v = threadIdx.x; v < (sizeof(T) == 1 ? 256 : 1024); v += 256) hist[v] = 0u;
        __syncthreads();
    }
    pyramid_tile<T, L>(sd, ss, local, lds, unary ? hist : nullptr);
    if (unary) store_tile_hist<T>(sd, local, hist);
}

// Unary intensity measure of each frame pyramided in the step (one 256-thread
// workgroup per frame, after k_pyramid): the frame histogram is the sum of its
// tile histograms (each thread adds 16-byte chunks of 8 bins over a strided
// subset of the tiles; the partial sums meet in LDS); then the exact sums and
// the three measures.  The workgroup is kept small (8 KB of LDS) so that it is
// placed at once next to the persistent motion-search grids: the ingest
// stream's next pyramid waits behind it.
constexpr int kIntThreads = 256;

__device__ __forceinline__ int64_t block_sum64_1024(int64_t v, int64_t* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();                               // red is free
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < kIntThreads / 64; ++w) t += red[w];
    return t;
}

__global__ void __launch_bounds__(kIntThreads) k_intensity(const StreamDesc* __restrict__ sds,
                                                          const StepStream* __restrict__ steps,
                                                          const int32_t* __restrict__ k1_list, int32_t n_k1) {
    __shared__ uint32_t part[8 * 256];             // [groups][bins]: 8 x 256 (8-bit) or 2 x 1024 (10-bit)
    __shared__ int64_t red[kIntThreads / 64];
    if ((int)blockIdx.x >= n_k1) return;
    const StepStream& ss = steps[k1_list[blockIdx.x]];
    const StreamDesc& sd = sds[ss.sid];
    if (!sd.tileh) return;
    const int nb = 1 << sd.bits, nt = ss.k1_tiles, tid = threadIdx.x;
    const int per = nb / 8, groups = kIntThreads / per;
    const int c = tid % per, g = tid / per;
    uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = g; t < nt; t += groups) {
        const uint4 q = reinterpret_cast<const uint4*>(sd.tileh + (int64_t)t * nb)[c];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[2 * k] += w[k] & 0xffffu;
            acc[2 * k + 1] += w[k] >> 16;
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) part[g * nb + 8 * c + k] = acc[k];
    __syncthreads();
    uint32_t* fh = reinterpret_cast<uint32_t*>(slot_base(sd, ss.frame) + sd.offH);
    int64_t n = 0, s1 = 0, s2 = 0;
    for (int v = tid; v < nb; v += kIntThreads) {
        uint32_t cnt = 0;
        for (int gg = 0; gg < groups; ++gg) cnt += part[gg * nb + v];
        part[v] = cnt;                             // group 0's row now holds the frame histogram
        fh[v] = cnt;
        n += cnt;
        s1 += (int64_t)v * cnt;
        s2 += (int64_t)v * v * cnt;
    }
    n = block_sum64_1024(n, red);
    s1 = block_sum64_1024(s1, red);
    s2 = block_sum64_1024(s2, red);
    int64_t m = 0;
    for (int v = tid; v < nb; v += kIntThreads) {
        const int64_t d = n * v - s1;
        m += (int64_t)part[v] * (d < 0 ? -d : d);
    }
    m = block_sum64_1024(m, red);
    if (tid == 0) {
        FrameInfo& fi = sd.info[ss.frame % sd.rs];
        fi.h_mean = (double)s1 / (double)n;
        fi.h_std = __builtin_sqrt((double)(n * s2 - s1 * s1)) / (double)n;
        fi.h_mad = (double)m / ((double)n * (double)n);
    }
}

hipError_t launch_intensity(const StreamDesc* sds, const StepStream* steps, const int32_t* k1_list, int32_t n_k1,
                            hipStream_t s) {
    if (n_k1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_intensity, dim3((unsigned)n_k1), dim3(kIntThreads), 0, s, sds, steps, k1_list, n_k1);
    return hipGetLastError();
}

int pyramid_tiles(const StreamDesc& sd) {
    return div_up(pyr_grid_w(sd), 16 * pyr_cw(sd.L)) * div_up(sd.hl[0], kPyrTH);
}

// Copy the step descriptor from mapped pinned host memory to device memory
// (one pass, 16-byte words); cheaper to enqueue than an API copy of the same size.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n = (bytes + 15) / 16;
    if (n <= 0) return hipSuccess;
    const int64_t grid = std::min<int64_t>((n + 255) / 256, 64);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const uint4*>(src),
                       reinterpret_cast<uint4*>(dst), n);
    return hipGetLastError();
}

// Launch the pyramid for one group of streams sharing sample width and L.
hipError_t launch_pyramid(int bits, int L, const StreamDesc* sds, const StepStream* steps, const int32_t* k1_list,
                          int32_t n_k1, int32_t total_tiles, TileJob* cjobs, int32_t* cmap, hipStream_t s,
                          LaunchTiming tm) {
    if (n_k1 <= 0 || total_tiles <= 0) return hipSuccess;
    const dim3 g(total_tiles), b(256);
#define VSA_PYR(TT, LL)                                                                                      \
    do {                                                                                                     \
        if (tm.any())                                                                                        \
            hipExtLaunchKernelGGL((k_pyramid<TT, LL>), g, b, 0, s, tm.start, tm.stop, 0, sds, steps, k1_list, \
                                  n_k1, cjobs, cmap);                                                        \
        else                                                                                                 \
            hipLaunchKernelGGL((k_pyramid<TT, LL>), g, b, 0, s, sds, steps, k1_list, n_k1, cjobs, cmap);     \
    } while (0)
    if (bits == 8) {
        switch (L) {
            case 0: VSA_PYR(uint8_t, 0); break;
            case 1: VSA_PYR(uint8_t, 1); break;
            case 2: VSA_PYR(uint8_t, 2); break;
            case 3: VSA_PYR(uint8_t, 3); break;
            default: VSA_PYR(uint8_t, 4); break;
        }
    } else {
        switch (L) {
            case 0: VSA_PYR(uint16_t, 0); break;
            case 1: VSA_PYR(uint16_t, 1); break;
            case 2: VSA_PYR(uint16_t, 2); break;
            case 3: VSA_PYR(uint16_t, 3); break;
            default: VSA_PYR(uint16_t, 4); break;
        }
    }
#undef VSA_PYR
    return hipGetLastError();
}

}  // namespace vsa
