// k_decide.hip -- K6: per-stream decision state machine, sparse-task compaction
// and record emission.
//
// The decisions are those of Sec. III.B-D: a fast check of the consecutive
// activity against the shot's recent history, a deep check of K-frame
// transitions (ACT from t to t+K against ACT from t back to its predecessor at
// the same distance, at a coarser pyramid level for larger K), the sampling
// structure vote over at most n_ss non-static frames of a shot from the field
// measures v0, v1, v2 (comb test, 3:2 pulldown cadence, field order from
// beta = v1/v2), and keyframes from the activity accumulated within a shot.
//
// Each stream advances one "iteration" of the offline sequential pass at a
// time, as soon as the frames it needs are on the device.  An iteration that
// needs sparse measures (fields of an analysed frame, deep-check pairs after
// the fast check fired) is planned in one step and committed in the next one,
// after the step's motion-search launch has computed the requested pairs;
// iterations that need nothing more are committed at once.  In the offline
// clip form (a field cache is given), an iteration that asks for the fields
// of its frame also asks for those of up to kMaxSpec later non-static frames
// already ingested, as many as the analysis window may still take; they are
// filed per ring slot under their frame, and a later iteration that wants a
// cached frame's fields commits without a new request.  The cached values are
// the same measures, so the records do not change.  The planned
// tasks of all streams are compacted into one dense list: each workgroup sums
// its streams' task and tile counts, reserves its slice of the list and of the
// tile range with one packed 64-bit atomic, hands each stream its offsets (a
// running sum over the workgroup's waves), and each stream writes its tasks
// there, with the running tile offsets that the persistent motion-search grid
// walks.  Finished frames and shots are appended to device output rings.
//
// All floating-point comparisons use the operations in the order written,
// with no contraction (-ffp-contract=off), so that the labels are bitwise
// reproducible against a scalar CPU implementation.
#include "vsa_internal.h"
#include "pair_finish.h"

namespace vsa {

namespace {

__device__ __forceinline__ int ceil_log2(int k) {
    int c = 0;
    while ((1 << c) < k) ++c;
    return c;
}

__device__ __forceinline__ int deep_level(const StreamDesc& sd, int K) {
    const int l = sd.L + ceil_log2(K);
    return l < sd.Lcap ? l : sd.Lcap;
}

__device__ __forceinline__ bool p_dup(const StreamDesc& sd, int K, int d);
__device__ __forceinline__ int p_rep(const StreamDesc& sd, int K, int d);

__device__ __forceinline__ FrameInfo& info_of(const StreamDesc& sd, int f) { return sd.info[f % sd.rs]; }

__device__ __forceinline__ void ss_reset(Analysis& a) {
    a.open = 1; a.n = 0; a.nci = 0; a.s = 0; a.result = 0; a.phase = -1;
    for (int i = 0; i < 5; ++i) { a.np[i] = 0; a.s0[i] = 0.0; }
    a.sum1 = 0.0; a.sum2 = 0.0;
}

// Per analysed frame: the interlace vote (v0 against the smaller of v1, v2:
// half a frame interval separates v0's fields and one of the inter-frame field
// pairs) and v0 summed per position of the 5-frame pulldown unit.
__device__ __forceinline__ void ss_add(Analysis& a, int ph, double v0, double v1, double v2,
                                       const DecideParams& dp) {
    const double mn = v1 < v2 ? v1 : v2;
    const bool comb_min = v0 > dp.tau_c * mn;
    a.n += 1;
#pragma unroll
    for (int q = 0; q < 5; ++q)
        if (q == ph) {
            a.np[q] += 1;
            a.s0[q] = a.s0[q] + v0;
        }
    if (comb_min) a.nci += 1;
    if (v1 > v2) a.s += 1; else if (v1 < v2) a.s -= 1;
    a.sum1 = a.sum1 + v1;
    a.sum2 = a.sum2 + v2;
}

__device__ __forceinline__ void ss_decide(Analysis& a, const DecideParams& dp) {
    a.open = 0;
    a.phase = -1;
    if (a.n == 0) { a.result = VSA_SAMPLING_UNDETERMINED; return; }
    if (a.n >= 10 && a.np[0] && a.np[1] && a.np[2] && a.np[3] && a.np[4]) {
        // 3:2 pulldown: mean v0 at positions q, q+1 above tau_p times the mean
        // at each other position (cross-multiplied; at most one q qualifies)
        for (int q = 0; q < 5; ++q) {
            const int b = q == 4 ? 0 : q + 1;
            bool ok = true;
            for (int r = 0; r < 5; ++r) {
                if (r == q || r == b) continue;
                const double rq = a.s0[r] * (double)a.np[q], rb = a.s0[r] * (double)a.np[b];
                ok = ok && (a.s0[q] * (double)a.np[r] > dp.tau_p * rq) && (a.s0[b] * (double)a.np[r] > dp.tau_p * rb);
            }
            if (ok) {
                a.result = VSA_SAMPLING_PULLDOWN32;
                a.phase = q;
                return;
            }
        }
    }
    bool inter;
    if ((double)a.nci <= dp.eps * (double)a.n) inter = false;
    else if ((double)a.nci >= (1.0 - dp.eps) * (double)a.n) inter = true;
    else inter = 2 * a.nci > a.n;
    if (!inter) { a.result = VSA_SAMPLING_PROGRESSIVE; return; }
    if (a.s > 0) a.result = VSA_SAMPLING_TFF;
    else if (a.s < 0) a.result = VSA_SAMPLING_BFF;
    else a.result = (a.sum1 >= a.sum2) ? VSA_SAMPLING_TFF : VSA_SAMPLING_BFF;
}

// Fast-check threshold from the recent activity of the shot (W_hist values,
// each capped at the threshold in force when it was pushed).
__device__ __forceinline__ double fast_thr(const DecideState& st, const DecideParams& dp) {
    if (st.hist_len == 0) return dp.theta_f0;       // no history in the shot yet
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxHist; ++i)              // oldest to newest
        if (i >= kMaxHist - st.hist_len) s = s + st.hist[i];
    const double mean = s / (double)st.hist_len;
    return dp.rho_f * mean + dp.theta_f;
}

__device__ __forceinline__ bool fast_check(const DecideState& st, double a, const DecideParams& dp) {
    return a > fast_thr(st, dp);
}

__device__ __forceinline__ void hist_push(DecideState& st, double a, const DecideParams& dp) {
#pragma unroll
    for (int i = 0; i < kMaxHist - 1; ++i) st.hist[i] = st.hist[i + 1];
    st.hist[kMaxHist - 1] = a;
    if (st.hist_len < dp.w_hist) st.hist_len += 1;
}

__device__ __forceinline__ void close_shot(DecideState& st, vsa_shot_result* closed, int last,
                                           const DecideParams& dp) {
    if (st.ss.open) ss_decide(st.ss, dp);
    if (st.n_closed >= kMaxClosed) return;
    vsa_shot_result& r = closed[st.n_closed++];
    r.shot_id = st.shot_id;
    r.pad0 = 0;
    r.first = st.shot_start;
    r.last = last;
    r.in_boundary = st.cur_in_boundary;
    r.in_k = st.cur_in_k;
    r.sampling = st.ss.result;
    r.pulldown_phase = st.ss.result == VSA_SAMPLING_PULLDOWN32 ? st.ss.phase : -1;
    r.n_analyzed = st.ss.n;
    r.final_ = 1;
}

// Deep check of iteration t from the requested results (Sec. III.B): K verifies
// when ACT(t, t+K) > rho_d * ACT(t, t-K) + theta_d; among the K with K and K+1
// verified, the first whose excess ACT(t, t+K) - ACT(t, t-K) reaches gamma of
// the largest excess is taken.
__device__ int deep_check(const StreamDesc& sd, const DecideState& st, int t, int Kn, double a_t,
                          const PairResult* res, const DecideParams& dp) {
    bool V[kMaxKmax + 3];
    double S[kMaxKmax + 3];
    for (int K = 0; K < kMaxKmax + 3; ++K) { V[K] = true; S[K] = 0.0; }
    for (int K = 1; K <= Kn; ++K) {
        const double f = K == 1 ? a_t : res[kResF + K].act;
        const int kp = min(K, t - st.shot_start);
        const double p = kp > 0 ? res[kResP + p_rep(sd, K, t - st.shot_start)].act : 0.0;
        V[K] = f > dp.rho_d * p + dp.theta_d;
        S[K] = f - p;
    }
    const int Kc = min(sd.k_max, Kn);
    bool any = false;
    double smax = 0.0;
    for (int K = 1; K <= Kc; ++K)
        if (V[K] && V[K + 1]) {
            if (!any || S[K] > smax) smax = S[K];
            any = true;
        }
    if (!any) return 0;
    for (int K = 1; K <= Kc; ++K)
        if (V[K] && V[K + 1] && S[K] >= dp.gamma * smax) return K;
    return 0;
}

// Commit iteration t = st.t with the flags it was planned with.
// a is the consecutive activity of t (the frame record's act).
__device__ void commit(const StreamDesc& sd, DecideState& st, vsa_shot_result* closed, const PairResult* res,
                       const DecideParams& dp, bool want_fields, bool fire, bool need_deep, int Kn, double a) {
    const int t = st.t;
    FrameInfo& fi = info_of(sd, t);
    if (want_fields) {
        const double v0 = res[kResFields + 0].act, v1 = res[kResFields + 1].act, v2 = res[kResFields + 2].act;
        fi.v[0] = v0; fi.v[1] = v1; fi.v[2] = v2;
        fi.field_mask = 7;
        fi.flags |= VSA_F_ANALYZED;
        ss_add(st.ss, (t - st.shot_start) % 5, v0, v1, v2, dp);
        if (st.ss.n == dp.n_ss) ss_decide(st.ss, dp);
    }
    if (fire) fi.flags |= VSA_F_FAST_FIRED;
    int Kstar = 0;
    if (need_deep) {
        Kstar = deep_check(sd, st, t, Kn, a, res, dp);
        if (!fire) Kstar = 0;
    }
    if (Kstar > 0) {
        fi.shot_id = st.shot_id;
        close_shot(st, closed, t, dp);
        for (int f = t + 1; f < t + Kstar; ++f) {
            FrameInfo& g = info_of(sd, f);
            g.flags |= VSA_F_IN_TRANSITION;
            g.shot_id = -1;
        }
        const int b = t + Kstar;
        FrameInfo& fb = info_of(sd, b);
        fb.boundary = Kstar == 1 ? 1 : 2;
        fb.boundary_k = Kstar;
        fb.flags |= VSA_F_SHOT_START | VSA_F_KEYFRAME;
        st.shot_id += 1;
        st.cur_in_boundary = fb.boundary;
        st.cur_in_k = Kstar;
        st.shot_start = b;
        st.hist_len = 0;
        st.acc = 0.0;
        ss_reset(st.ss);
        st.t = b;
        return;
    }
    fi.shot_id = st.shot_id;
    hist_push(st, fire ? fast_thr(st, dp) : a, dp);
    st.acc = st.acc + a;
    if (st.acc > dp.theta_kf) {
        info_of(sd, t + 1).flags |= VSA_F_KEYFRAME;
        st.acc = 0.0;
    }
    st.t = t + 1;
}

// Backward deep-check pairs: for K beyond the shot start (K' = t - shot_start
// < K) the pair t -> t-K' repeats; at the same pyramid level it is the same
// measure, computed once (the first such K) and shared.
__device__ __forceinline__ bool p_dup(const StreamDesc& sd, int K, int d) {
    return K > d && K - 1 >= d && deep_level(sd, K - 1) == deep_level(sd, K);
}

__device__ __forceinline__ int p_rep(const StreamDesc& sd, int K, int d) {
    while (p_dup(sd, K, d)) --K;
    return K;
}

// Sparse tasks of the planned iteration, in a fixed order: v0, v1, v2, then
// F_K for K = 2..Kn, then the distinct P_K for K = 1..Kn (when t > shot start).
// Speculative field tasks (three per frame of st.spec_mask) follow them.
__device__ __forceinline__ int plan_regular_count(const StreamDesc& sd, const DecideState& st) {
    int n = st.plan_nf ? 3 : 0;
    if (st.plan_deep) {
        n += st.plan_kn - 1;
        const int d = st.t - st.shot_start;
        if (d > 0)
            for (int K = 1; K <= st.plan_kn; ++K) n += p_dup(sd, K, d) ? 0 : 1;
    }
    return n;
}

template <bool kSpec>
__device__ __forceinline__ int plan_task_count(const StreamDesc& sd, const DecideState& st) {
    if (!st.plan) return 0;
    return plan_regular_count(sd, st) + (kSpec ? 3 * st.plan_spec : 0);
}

// The three field pairs of frame u (Sec. III.C): v0 = (U_u, D_u),
// v1 = (U_u, D_u+1), v2 = (D_u, U_u+1).
__device__ __forceinline__ void field_task(const StreamDesc& sd, int u, int i, PairTask& k) {
    k.kind = MK_FIELD;
    k.ref = u;
    k.ref_field = (i == 2) ? PL_LOWER : PL_UPPER;
    k.oth = (i == 0) ? u : u + 1;
    k.oth_field = (i == 2) ? PL_UPPER : PL_LOWER;
    k.level = sd.Lf;
    k.tiles = field_pair_tiles(sd.search, sd.wf, sd.hf);
}

template <bool kSpec>
__device__ PairTask plan_task(const StreamDesc& sd, const DecideState& st, int sid, int i) {
    PairTask k;
    k.sid = sid;
    k.flags = 0;
    k.epoch = sd.epoch;
    k.tile_prefix = 0;
    const int t = st.t;
    if (kSpec && st.plan_spec > 0) {
        const int reg = plan_regular_count(sd, st);
        if (i >= reg) {
            const int j = (i - reg) / 3, c = (i - reg) % 3;
            uint32_t m = st.spec_mask;
            for (int q = 0; q < j; ++q) m &= m - 1;       // drop the j lowest frames
            field_task(sd, t + 1 + __builtin_ctz(m), c, k);
            k.result = kResSpec + c;
            return k;
        }
    }
    if (st.plan_nf) {
        if (i < 3) {
            field_task(sd, t, i, k);
            k.result = kResFields + i;
            return k;
        }
        i -= 3;
    }
    const int nF = st.plan_kn - 1;
    if (i < nF) {
        const int K = i + 2;
        k.kind = MK_DEEP_F;
        k.ref = t; k.ref_field = PL_FRAME;
        k.oth = t + K; k.oth_field = PL_FRAME;
        k.level = deep_level(sd, K);
        k.result = kResF + K;
    } else {
        const int d = t - st.shot_start;
        int j = i - nF, K = 1;
        for (;; ++K) {
            if (!p_dup(sd, K, d)) {
                if (j == 0) break;
                --j;
            }
        }
        const int kp = min(K, d);
        k.kind = MK_DEEP_P;
        k.ref = t; k.ref_field = PL_FRAME;
        k.oth = t - kp; k.oth_field = PL_FRAME;
        k.level = deep_level(sd, K);
        k.result = kResP + K;
    }
    const int dl = k.level - sd.L;
    k.tiles = frame_pair_tiles(sd.search, sd.wl[dl], sd.hl[dl]);
    return k;
}

struct PlaneDims { int w, h; };

__device__ __forceinline__ PlaneDims plane_dims(const StreamDesc& sd, const PairTask& t) {
    if (t.ref_field != PL_FRAME) return PlaneDims{sd.wf, sd.hf};
    const int d = t.level - sd.L;
    return PlaneDims{sd.wl[d], sd.hl[d]};
}

// Cached speculative fields of frame u into the result slots of an
// iteration's own field measures; false if u's are not cached.
__device__ __forceinline__ bool spec_fetch(const StreamDesc& sd, int u, PairResult* res, const DecideParams& dp) {
    const double* cv = dp.spec + (int64_t)(u % sd.rs) * 4;
    if (!(cv[3] == (double)u)) return false;
    for (int i = 0; i < 3; ++i) { res[kResFields + i].act = cv[i]; res[kResFields + i].swr = 0.0; }
    return true;
}

// Consecutive activity and static bit of frames base .. base+n-1, staged in
// LDS by the whole wave before a long sequential pass (both are final before
// the pass runs, which only reads them); act == nullptr: none staged.
struct Staged {
    const double* act;
    const uint8_t* stat;
    int base, n;
};

__device__ __forceinline__ double act_at(const StreamDesc& sd, const Staged& pf, int f) {
    const int k = f - pf.base;
    if (pf.act && k >= 0 && k < pf.n) return pf.act[k];
    return info_of(sd, f).act;
}

__device__ __forceinline__ bool static_at(const StreamDesc& sd, const Staged& pf, int f) {
    const int k = f - pf.base;
    if (pf.act && k >= 0 && k < pf.n) return pf.stat[k] != 0;
    return (info_of(sd, f).flags & VSA_F_STATIC) != 0;
}

__device__ __forceinline__ void log_task(int32_t* log, int64_t cap, DecideState& st, const PairTask& k);

// Advance one stream as far as the ingested frames allow (kSpec: with the
// speculative field measures when dp.spec is given).  A frame whose fields
// the pass takes from the speculative cache counts (and is logged, with
// slog) as the three field measures it requested.
template <bool kSpec>
__device__ void advance(const StreamDesc& sd, DecideState& st, vsa_shot_result* closed, PairResult* res,
                        const DecideParams& dp, int has_frame, int frame, int ended_T, const Staged& pf,
                        int32_t* slog = nullptr, int64_t log_cap = 0) {
    st.n_closed = 0;
    if (st.done) { st.plan = 0; return; }
    if (has_frame) st.n = frame;
    if (ended_T >= 0) st.T_end = ended_T;
    const bool spec_on = kSpec && dp.spec != nullptr && !dp.dense;
    if (st.plan) {
        // fields wanted but not requested: they were in the cache when planned
        if (spec_on && st.plan_want && !st.plan_nf) spec_fetch(sd, st.t, res, dp);
        commit(sd, st, closed, res, dp, st.plan_want, st.plan_fire, st.plan_deep, st.plan_kn, act_at(sd, pf, st.t));
        st.plan = 0;
    }
    for (;;) {
        const int t = st.t;
        if (st.T_end >= 0 && t >= st.T_end - 1) {
            if (st.T_end > 0) {
                info_of(sd, st.T_end - 1).shot_id = st.shot_id;
                close_shot(st, closed, st.T_end - 1, dp);
            }
            st.t = st.T_end;
            st.done = 1;
            break;
        }
        if (t + 1 > st.n) break;                  // pair t -> t+1 not finished yet
        const double a = act_at(sd, pf, t);
        const bool stat = static_at(sd, pf, t);
        const bool want = st.ss.open && !stat;    // static frames carry no information
        const bool fire = fast_check(st, a, dp);
        const bool need_fields = want || dp.dense;
        const bool need_deep = fire || dp.dense;
        int Kn = 0;
        if (need_deep) {
            if (st.T_end >= 0) Kn = min(sd.k_max + 1, st.T_end - 1 - t);
            else if (t + sd.k_max + 1 <= st.n) Kn = sd.k_max + 1;
            else break;                           // wait for the look-ahead frames
        }
        const bool cached = spec_on && want && spec_fetch(sd, t, res, dp);
        if (cached)
            for (int i = 0; i < 3; ++i) {
                PairTask k;
                field_task(sd, t, i, k);
                log_task(slog, log_cap, st, k);
            }
        st.plan_want = want;
        st.plan_fire = fire;
        st.plan_deep = need_deep;
        st.plan_nf = need_fields && !cached;
        st.plan_kn = Kn;
        st.plan_spec = 0;
        st.spec_mask = 0;
        st.plan = 1;
        if (spec_on && st.plan_nf && !need_deep) {
            // the fields of the next non-static frames already ingested, as
            // many as the analysis window may still take: computed with t's
            int quota = dp.n_ss - st.ss.n - 1;
            // (frames below spec_next were planned before, or skipped as
            // static: the cache check in the pass covers them either way)
            for (int k = 0; k < 32 && t + 1 + k + 1 <= st.n && quota > 0 && st.plan_spec < kMaxSpec; ++k) {
                const int u = t + 1 + k;
                if (static_at(sd, pf, u)) continue;
                --quota;
                if (u < st.spec_next) continue;
                st.spec_mask |= 1u << k;
                st.plan_spec += 1;
                st.spec_next = u + 1;
            }
        }
        if (plan_task_count<kSpec>(sd, st) > 0) break;       // measures requested; commit next step
        st.plan = 0;
        commit(sd, st, closed, res, dp, want, fire, need_deep, Kn, a);
    }
}

__device__ void fill_record(vsa_frame_result& r, const FrameInfo& fi) {
    r.frame = fi.frame;
    r.pts = fi.pts;
    r.flags = fi.flags;
    r.shot_id = fi.shot_id;
    r.boundary = fi.boundary;
    r.boundary_k = fi.boundary_k;
    r.ncc = fi.ncc; r.swr = fi.swr; r.amm = fi.amm; r.act = fi.act;
    for (int k = 0; k < 5; ++k) r.mom[k] = fi.mom[k];
    r.n_pix = fi.n_pix;
    r.amm_num = fi.amm_num;
    r.n_blocks = fi.n_blocks;
    r.field_mask = fi.field_mask;
    r.v[0] = fi.v[0]; r.v[1] = fi.v[1]; r.v[2] = fi.v[2];
    r.h_mean = fi.h_mean; r.h_std = fi.h_std; r.h_mad = fi.h_mad;
}

__device__ __forceinline__ void log_task(int32_t* log, int64_t cap, DecideState& st, const PairTask& k) {
    if (log && st.log_count < cap) {
        int32_t* e = log + 6 * st.log_count;
        e[0] = k.kind; e[1] = k.ref; e[2] = k.oth; e[3] = k.ref_field; e[4] = k.oth_field; e[5] = k.level;
    }
    st.log_count += 1;
}

}  // namespace

__device__ __forceinline__ int64_t wsum64(int64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wavefront per stream (eight per workgroup), after the step's motion search:
//  1. the wave sums the tile partials of the stream's consecutive pair and
//     lane 0 finishes it (NCC, SWR, AMM, ACT) into the frame's record;
//  2. likewise for each sparse pair the stream planned last step, into the
//     wave's result slots in LDS;
//  3. lane 0 advances the stream's state machine with descriptor and state in
//     registers, reserves its slice of the next step's sparse task list (tasks
//     and tiles from one 64-bit atomic, so tile offsets grow with task order)
//     and of the output rings, and writes its tasks;
//  4. the wave copies the finished frame and shot records out in parallel.
// Streams never share a wave, so their control paths do not serialise.
template <bool kSpec>
__global__ void __launch_bounds__(64 * kDecideWaves) k_finish_decide(
    const StreamDesc* __restrict__ sds, DecideState* __restrict__ states, const StepStream* __restrict__ steps,
    int32_t n_steps, DecideParams dp, const TilePartial* __restrict__ cpart, const TilePartial* __restrict__ spart,
    const PairTask* __restrict__ sparse_prev, PairTask* __restrict__ sparse_next, DeviceCursors* __restrict__ cur,
    OutFrame* __restrict__ out_frames, uint64_t frames_cap, OutShot* __restrict__ out_shots, uint64_t shots_cap,
    int32_t* __restrict__ log, int64_t log_cap, vsa_shot_result* __restrict__ closed_buf, int32_t par,
    PubSnap* __restrict__ snap, TileJob* __restrict__ sjobs_next, int32_t* __restrict__ smap_next) {
    struct Bcast {
        FrameInfo* info;
        int32_t rs, sid, epoch, e0, nframes, nshots, ntasks, tiles, blocks;
        uint64_t fbase, sbase;
        int32_t task, tile;
    };
    __shared__ Bcast bc[kDecideWaves];
    __shared__ PairResult res[kDecideWaves][kResSlots];
    constexpr int kMaxT = 3 + 2 * (kMaxKmax + 1);
    __shared__ int32_t tpre[kDecideWaves][kMaxT];
    __shared__ int32_t npre[kDecideWaves][kMaxT + 1];   // first tile of each planned task, then the end
    // the decisions are on the critical path of every step while other
    // streams' motion search shares the CUs: their waves issue first
    __builtin_amdgcn_s_setprio(3);
    __shared__ int64_t acc[kDecideWaves][kMaxT][6];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * kDecideWaves + wave;
    const bool active = i < n_steps;
    StepStream ss;
    int sid = -1;
    if (active) {
        ss = steps[i];
        sid = ss.sid;
        const StreamDesc& sd = sds[sid];
        // 1. consecutive pair (frame-1 -> frame) of this step: lanes stride over its tiles
        if (ss.has_frame && ss.consec_tiles > 0 && sd.search == 2) {
            // the dense flow: the pair's tiles hold its row sums
            const FlowFinish f = flow_finish(reinterpret_cast<const FlowRow*>(cpart + ss.consec_prefix), sd.wl[0],
                                             sd.hl[0], dp.a0, dp.a_static_fx);
            if (lane == 0) {
                FrameInfo& fi = sd.info[(ss.frame - 1) % sd.rs];
                fi.ncc = f.ncc; fi.swr = f.swr; fi.amm = f.amm; fi.act = f.act;
                for (int k = 0; k < 5; ++k) fi.mom[k] = 0;
                fi.n_pix = (int64_t)sd.wl[0] * sd.hl[0];
                fi.amm_num = 0;
                fi.n_blocks = 0;
                fi.flags |= VSA_F_HAS_PAIR | (f.is_static ? VSA_F_STATIC : 0);
            }
        } else if (ss.has_frame && ss.consec_tiles > 0) {
            int64_t a[6] = {0, 0, 0, 0, 0, 0};
            for (int q = lane; q < ss.consec_tiles; q += 64) {
                const TilePartial& p = cpart[ss.consec_prefix + q];
                a[0] += p.sx; a[1] += p.sy; a[2] += p.sxx; a[3] += p.syy; a[4] += p.sxy; a[5] += p.a;
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) a[k] = wsum64(a[k]);
            if (lane == 0) {
                const int64_t B = sd.B_L, n = 64 * B;
                double f[4];
                finish_pair(a[0], a[1], a[2], a[3], a[4], n, a[5], B, dp.a0, f);
                FrameInfo& fi = sd.info[(ss.frame - 1) % sd.rs];
                fi.ncc = f[0]; fi.swr = f[1]; fi.amm = f[2]; fi.act = f[3];
                for (int k = 0; k < 5; ++k) fi.mom[k] = a[k];
                fi.n_pix = n;
                fi.amm_num = a[5];
                fi.n_blocks = (int32_t)B;
                fi.flags |= VSA_F_HAS_PAIR | (a[5] < (int64_t)dp.a_static_fx * B ? VSA_F_STATIC : 0);
            }
        }
        // 2. sparse pairs planned by the previous step.  A stream's tasks are
        //    contiguous in the list and so are their tiles: the lanes stride
        //    over the whole tile range once, add each partial to its task's
        //    LDS accumulators, and lane j then finishes task j.
        const int spb = states[sid].sp_base, spc = states[sid].sp_count;
        PairTask mine;
        mine.tiles = 0;
        if (lane < spc) {
            mine = sparse_prev[spb + lane];
            tpre[wave][lane] = mine.tile_prefix;
            for (int k = 0; k < 6; ++k) acc[wave][lane][k] = 0;
        }
        if (spc > 0 && sd.search == 2) {
            // the dense flow: task by task, the whole wave adds up its row sums
            for (int j = 0; j < spc; ++j) {
                const PairTask tk = sparse_prev[spb + j];
                if (tk.epoch != sd.epoch || tk.result < 0) continue;
                const PlaneDims pd = plane_dims(sd, tk);
                const FlowFinish f = flow_finish(reinterpret_cast<const FlowRow*>(spart + tk.tile_prefix), pd.w, pd.h,
                                                 dp.a0, dp.a_static_fx);
                if (lane != 0) continue;
                if (kSpec && tk.result >= kResSpec) {
                    double* cv = dp.spec + (int64_t)(tk.ref % sd.rs) * 4;
                    cv[tk.result - kResSpec] = f.act;
                    cv[3] = (double)tk.ref;
                } else {
                    res[wave][tk.result].act = f.act;
                    res[wave][tk.result].swr = f.swr;
                }
            }
        } else if (spc > 0) {
            // each lane takes one contiguous run of the tile range: its loads
            // are independent (many in flight), it sums each task's part of
            // the run in registers and adds it to the task's accumulators
            // once (a run spans few tasks, so the LDS atomics rarely collide)
            const int t0 = __shfl(mine.tile_prefix, 0, 64);
            const int t_last = __shfl(mine.tile_prefix + mine.tiles, spc - 1, 64);
            const int per = (t_last - t0 + 63) / 64;
            int q = t0 + lane * per;
            const int q_end = min(t_last, q + per);
            if (q < q_end) {
                int j = 0, hi = spc - 1;        // last task whose first tile is <= q
                while (j < hi) {
                    const int mid = (j + hi + 1) >> 1;
                    if (tpre[wave][mid] <= q) j = mid; else hi = mid - 1;
                }
                while (q < q_end) {
                    const int seg_end = min(q_end, j + 1 < spc ? tpre[wave][j + 1] : t_last);
                    int64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
#pragma unroll 8
                    for (; q < seg_end; ++q) {
                        const TilePartial& p = spart[q];
                        s0 += p.sx; s1 += p.sy; s2 += p.sxx; s3 += p.syy; s4 += p.sxy; s5 += p.a;
                    }
                    unsigned long long* acc_t = reinterpret_cast<unsigned long long*>(acc[wave][j]);
                    atomicAdd(acc_t + 0, (unsigned long long)s0);
                    atomicAdd(acc_t + 1, (unsigned long long)s1);
                    atomicAdd(acc_t + 2, (unsigned long long)s2);
                    atomicAdd(acc_t + 3, (unsigned long long)s3);
                    atomicAdd(acc_t + 4, (unsigned long long)s4);
                    atomicAdd(acc_t + 5, (unsigned long long)s5);
                    ++j;
                }
            }
        }
        if (lane < spc && mine.epoch == sd.epoch && mine.result >= 0 && sd.search != 2) {
            const int64_t* a = acc[wave][lane];
            int w, h;
            if (mine.ref_field != PL_FRAME) { w = sd.wf; h = sd.hf; }
            else { w = sd.wl[mine.level - sd.L]; h = sd.hl[mine.level - sd.L]; }
            const int64_t B = (int64_t)(w / kBlock) * (h / kBlock), n = 64 * B;
            double f[4];
            finish_pair(a[0], a[1], a[2], a[3], a[4], n, a[5], B, dp.a0, f);
            if (kSpec && mine.result >= kResSpec) {   // a speculative field measure: into the cache
                double* cv = dp.spec + (int64_t)(mine.ref % sd.rs) * 4;
                cv[mine.result - kResSpec] = f[3];
                cv[3] = (double)mine.ref;
            } else {
                res[wave][mine.result].act = f[3];
                res[wave][mine.result].swr = f[1];
            }
        }
    }
    __syncthreads();
    // With speculation (the offline clip form: one stream, whose pass may
    // run over a whole chunk in this launch), the wave stages the activity
    // and static bit of the frames the pass can reach into LDS, so that its
    // lane-0 loop does not wait on a global load per frame.
    constexpr int kPf = kSpec ? 512 : 1;
    __shared__ double pf_act[kDecideWaves][kPf];
    __shared__ uint8_t pf_stat[kDecideWaves][kPf];
    int pf_base = 0, pf_n = 0;
    if (kSpec && active) {
        const StreamDesc& sg = sds[sid];
        pf_base = states[sid].t;
        const int newest = ss.has_frame ? ss.frame : states[sid].n;
        pf_n = max(0, min(kPf, newest + 1 - pf_base));
        for (int k = lane; k < pf_n; k += 64) {
            const FrameInfo& fi = sg.info[(pf_base + k) % sg.rs];
            pf_act[wave][k] = fi.act;
            pf_stat[wave][k] = (fi.flags & VSA_F_STATIC) ? 1 : 0;
        }
    }
    __syncthreads();
    // 3. decisions (lane 0 of each wave), counts of what the stream produces.
    //    The descriptor is copied to LDS: a private copy, indexed by pyramid
    //    level at run time, would live in scratch, and reads in place would
    //    be repeated after every store of a planned task (the compiler cannot
    //    tell them apart).
    __shared__ StreamDesc sd_lds[kDecideWaves];
    const StreamDesc& sd = sd_lds[wave];
    // with speculation (up to 3 + 3 kMaxSpec tasks a launch) the planned
    // tasks are sized and written one lane per task from an LDS copy of the
    // decision state; otherwise lane 0 does it
    __shared__ DecideState st_lds[kSpec ? kDecideWaves : 1];
    __shared__ int32_t ptile[kSpec ? kDecideWaves : 1][kMaxT], pblk[kSpec ? kDecideWaves : 1][kMaxT];
    DecideState st;
    if (active && lane == 0) {
        sd_lds[wave] = sds[sid];
        st = states[sid];
        vsa_shot_result* closed = closed_buf + (int64_t)sid * kMaxClosed;
        const int e0 = st.emitted;
        const Staged pf{kSpec ? pf_act[wave] : nullptr, kSpec ? pf_stat[wave] : nullptr, pf_base, pf_n};
        advance<kSpec>(sd, st, closed, res[wave], dp, ss.has_frame, ss.frame, ss.ended_T, pf,
                       kSpec && log ? log + (int64_t)sid * log_cap * 6 : nullptr, log_cap);
        const int nt = plan_task_count<kSpec>(sd, st);
        int tiles = 0, blocks = 0;
        if (kSpec) {
            st_lds[wave] = st;
        } else {
            for (int q = 0; q < nt; ++q) {
                const PairTask pt = plan_task<kSpec>(sd, st, sid, q);
                tiles += pt.tiles;
                const PlaneDims pd = plane_dims(sd, pt);
                blocks += (pd.w / kBlock) * (pd.h / kBlock);
            }
        }
        Bcast& b = bc[wave];
        b.info = sd.info; b.rs = sd.rs; b.sid = sid; b.epoch = sd.epoch; b.e0 = e0; b.nframes = st.t - e0; b.nshots = st.n_closed;
        b.ntasks = nt; b.tiles = tiles; b.blocks = blocks;
    } else if (lane == 0) {
        Bcast& b = bc[wave];
        b.nframes = 0; b.nshots = 0; b.ntasks = 0; b.tiles = 0; b.blocks = 0;
    }
    __syncthreads();
    if (kSpec) {
        // tiles and blocks of the planned tasks, one lane per task
        if (active && lane < bc[wave].ntasks) {
            const PairTask pt = plan_task<kSpec>(sd, st_lds[wave], sid, lane);
            const PlaneDims pd = plane_dims(sd, pt);
            ptile[wave][lane] = pt.tiles;
            pblk[wave][lane] = (pd.w / kBlock) * (pd.h / kBlock);
        }
        __syncthreads();
        if (active && lane == 0) {
            int tiles = 0, blocks = 0;
            for (int q = 0; q < bc[wave].ntasks; ++q) { tiles += ptile[wave][q]; blocks += pblk[wave][q]; }
            bc[wave].tiles = tiles;
            bc[wave].blocks = blocks;
        }
        __syncthreads();
    }
    // one reservation per counter for the whole workgroup
    if (threadIdx.x == 0) {
        int nt = 0, ti = 0, nf = 0, ns = 0, bl = 0;
        for (int w = 0; w < kDecideWaves; ++w) {
            nt += bc[w].ntasks; ti += bc[w].tiles; nf += bc[w].nframes; ns += bc[w].nshots; bl += bc[w].blocks;
        }
        const unsigned long long rsv =
            nt ? atomicAdd(&cur->sparse_tt[par].v, ((unsigned long long)nt << 32) | (unsigned long long)ti) : 0ull;
        const unsigned long long fb = nf ? atomicAdd(&cur->frames_written.v, (unsigned long long)nf) : 0ull;
        const unsigned long long sb = ns ? atomicAdd(&cur->shots_written.v, (unsigned long long)ns) : 0ull;
        if (nt) {
            atomicAdd(&cur->sparse_run.v, (unsigned long long)nt);
            atomicAdd(&cur->sparse_blocks.v, (unsigned long long)bl);
        }
        int task = tt_tasks(rsv), tile = tt_tiles(rsv);
        uint64_t f = fb, s2 = sb;
        for (int w = 0; w < kDecideWaves; ++w) {
            bc[w].task = task; bc[w].tile = tile; bc[w].fbase = f; bc[w].sbase = s2;
            task += bc[w].ntasks; tile += bc[w].tiles; f += bc[w].nframes; s2 += bc[w].nshots;
        }
    }
    __syncthreads();
    if (kSpec && active && lane < bc[wave].ntasks) {
        // task `lane`: its first tile follows the tiles of the tasks before it
        const Bcast& b = bc[wave];
        int pre = b.tile;
        for (int r = 0; r < lane; ++r) pre += ptile[wave][r];
        PairTask t = plan_task<kSpec>(sd, st_lds[wave], sid, lane);
        t.tile_prefix = pre;
        sparse_next[b.task + lane] = t;
        sjobs_next[b.task + lane] = make_tile_job(sd, t, nullptr);
        npre[wave][lane] = pre;
    }
    if (kSpec && active && lane == 0) {
        const Bcast& b = bc[wave];
        int32_t* slog = log ? log + (int64_t)sid * log_cap * 6 : nullptr;
        int end = b.tile;
        const int regular = b.ntasks > 0 ? plan_regular_count(sd, st) : 0;
        for (int q = 0; q < b.ntasks; ++q) {
            end += ptile[wave][q];
            // the measures the pass asked for; speculative ones are only counted
            if (q < regular) log_task(slog, log_cap, st, plan_task<kSpec>(sd, st, sid, q));
        }
        st.spec_count += b.ntasks - regular;
        npre[wave][b.ntasks] = end;
        st.sp_base = b.task;
        st.sp_count = b.ntasks;
        st.emitted = st.t;
        states[sid] = st;
    }
    if (!kSpec && active && lane == 0) {
        const Bcast& b = bc[wave];
        int32_t* slog = log ? log + (int64_t)sid * log_cap * 6 : nullptr;
        int tile = b.tile;
        for (int q = 0; q < b.ntasks; ++q) {
            PairTask t = plan_task<kSpec>(sd, st, sid, q);
            t.tile_prefix = tile;
            tile += t.tiles;
            sparse_next[b.task + q] = t;
            // the next step's motion search finds the task's tiles through the
            // job and the tile map (filled by the whole wave below)
            sjobs_next[b.task + q] = make_tile_job(sd, t, nullptr);
            npre[wave][q] = t.tile_prefix;
            log_task(slog, log_cap, st, t);
        }
        npre[wave][b.ntasks] = tile;
        st.sp_base = b.task;
        st.sp_count = b.ntasks;
        st.emitted = st.t;
        states[sid] = st;
    }
    __syncthreads();
    // 4. tile map of the planned tasks and records out, the whole wave
    if (active) {
        const Bcast& b = bc[wave];
        if (b.ntasks > 0) {
            const int t_end = npre[wave][b.ntasks];
            int q = 0;
            for (int tt = b.tile + lane; tt < t_end; tt += 64) {
                while (q + 1 < b.ntasks && npre[wave][q + 1] <= tt) ++q;   // tiles ascend with the lane stride
                smap_next[tt] = b.task + q;
            }
        }
        for (int q = lane; q < b.nframes; q += 64) {
            OutFrame& o = out_frames[(b.fbase + (uint64_t)q) % frames_cap];
            o.sid = b.sid;
            o.pad = b.epoch;   // lets the host drop records of a slot's earlier stream
            fill_record(o.r, b.info[(b.e0 + q) % b.rs]);
        }
        if (lane < b.nshots) {
            OutShot& o = out_shots[(b.sbase + (uint64_t)lane) % shots_cap];
            o.sid = b.sid;
            o.pad = b.epoch;   // lets the host drop records of a slot's earlier stream
            o.r = closed_buf[(int64_t)b.sid * kMaxClosed + lane];
        }
    }
    // 5. the last workgroup to finish publishes the step's cursors: every
    //    reservation (and every record) of the step precedes its count
    __syncthreads();
    if (snap && threadIdx.x == 0) {
        __threadfence();
        const unsigned long long done = atomicAdd(&cur->blocks_done.v, 1ull);
        if (done == (unsigned long long)gridDim.x - 1) {
            __threadfence();
            PubSnap p;
            p.frames_written = atomicAdd(&cur->frames_written.v, 0ull);
            p.shots_written = atomicAdd(&cur->shots_written.v, 0ull);
            p.sparse_run = atomicAdd(&cur->sparse_run.v, 0ull);
            p.sparse_blocks = atomicAdd(&cur->sparse_blocks.v, 0ull);
            *snap = p;
            atomicExch(&cur->blocks_done.v, 0ull);
        }
    }
}

// Decision logic alone on injected measures: simulates one frame arrival per
// step, fills each planned task's result from the injected arrays (as the
// motion-search launch would), and writes the records and the task log.
__global__ void k_decide_replay(StreamDesc sd, DecideState* st_, PairResult* res, DecideParams dp, int32_t T,
                                const double* act, const double* swr, const uint8_t* stat, const double* v,
                                const double* F, const double* S, const double* P,
                                vsa_frame_result* recs, vsa_shot_result* shots, int32_t shots_cap,
                                int32_t* n_shots, int32_t* log, int32_t log_cap, int32_t* n_log) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DecideState st = *st_;
    vsa_shot_result closed[kMaxClosed];
    const int kw = sd.k_max + 2;
    int ns = 0;
    int nl = 0;
    const double nan = __builtin_nan("");
    for (int step = 0; step < T + 4 * (sd.k_max + 4) && !st.done; ++step) {
        const int has = step < T;
        if (has) {
            FrameInfo& fi = info_of(sd, step);
            fi.frame = step; fi.pts = step;
            fi.flags = step == 0 ? (VSA_F_KEYFRAME | VSA_F_SHOT_START) : 0;
            fi.shot_id = -1; fi.boundary = 0; fi.boundary_k = 0;
            fi.ncc = fi.swr = fi.amm = fi.act = nan;
            for (int k = 0; k < 5; ++k) fi.mom[k] = 0;
            fi.n_pix = 0; fi.amm_num = 0; fi.n_blocks = 0; fi.field_mask = 0;
            fi.v[0] = fi.v[1] = fi.v[2] = nan;
            if (step >= 1) {
                FrameInfo& pi = info_of(sd, step - 1);
                pi.act = act[step - 1];
                pi.swr = swr[step - 1];
                pi.ncc = 1.0 - swr[step - 1];
                pi.flags |= VSA_F_HAS_PAIR | (stat[step - 1] ? VSA_F_STATIC : 0);
            }
        }
        const int e0 = st.emitted;
        advance<false>(sd, st, closed, res, dp, has, step, step >= T - 1 ? T : -1, Staged{nullptr, nullptr, 0, 0});
        for (int f = e0; f < st.t; ++f) fill_record(recs[f], info_of(sd, f));
        st.emitted = st.t;
        for (int k = 0; k < st.n_closed; ++k)
            if (ns < shots_cap) shots[ns++] = closed[k];
        const int nt = plan_task_count<false>(sd, st);
        for (int k = 0; k < nt; ++k) {
            const PairTask t = plan_task<false>(sd, st, 0, k);
            if (log && nl < log_cap) {
                int32_t* e = log + 6 * nl;
                e[0] = t.kind; e[1] = t.ref; e[2] = t.oth; e[3] = t.ref_field; e[4] = t.oth_field;
                e[5] = t.kind == MK_FIELD ? -1 : t.level - sd.L;
            }
            ++nl;
            const int tt = st.t;
            PairResult& r = res[t.result];
            if (t.kind == MK_FIELD) { r.act = v[(int64_t)tt * 3 + (t.result - kResFields)]; r.swr = 0.0; }
            else if (t.kind == MK_DEEP_F) {
                const int K = t.result - kResF;
                r.act = F[(int64_t)tt * kw + K]; r.swr = S[(int64_t)tt * kw + K];
            } else {
                const int K = t.result - kResP;
                r.act = P[(int64_t)tt * kw + K]; r.swr = 0.0;
            }
        }
    }
    *n_shots = ns;
    *n_log = nl;
    *st_ = st;
}

hipError_t launch_finish_decide(const StreamDesc* sds, DecideState* states, const StepStream* steps, int32_t n_steps,
                                const DecideParams& dp, const TilePartial* cpart, const TilePartial* spart,
                                const PairTask* sparse_prev, PairTask* sparse_next, DeviceCursors* cur,
                                OutFrame* out_frames, uint64_t frames_cap, OutShot* out_shots, uint64_t shots_cap,
                                int32_t* log, int64_t log_cap, vsa_shot_result* closed_buf, int32_t par,
                                PubSnap* snap, TileJob* sjobs_next, int32_t* smap_next, hipStream_t s,
                                LaunchTiming tm) {
    if (n_steps <= 0) return hipSuccess;
    const dim3 g((n_steps + kDecideWaves - 1) / kDecideWaves), b(64 * kDecideWaves);
#define VSA_K6(SPEC)                                                                                            \
    do {                                                                                                        \
        if (tm.any())                                                                                           \
            hipExtLaunchKernelGGL(k_finish_decide<SPEC>, g, b, 0, s, tm.start, tm.stop, 0, sds, states, steps,  \
                                  n_steps, dp, cpart, spart, sparse_prev, sparse_next, cur, out_frames,         \
                                  frames_cap, out_shots, shots_cap, log, log_cap, closed_buf, par, snap,        \
                                  sjobs_next, smap_next);                                                       \
        else                                                                                                    \
            hipLaunchKernelGGL(k_finish_decide<SPEC>, g, b, 0, s, sds, states, steps, n_steps, dp, cpart,       \
                               spart, sparse_prev, sparse_next, cur, out_frames, frames_cap, out_shots,         \
                               shots_cap, log, log_cap, closed_buf, par, snap, sjobs_next, smap_next);          \
    } while (0)
    if (dp.spec) VSA_K6(true);
    else VSA_K6(false);
#undef VSA_K6
    return hipGetLastError();
}

hipError_t launch_decide_replay(const StreamDesc& sd, DecideState* st, PairResult* res, const DecideParams& dp,
                                int32_t T, const double* act, const double* swr, const uint8_t* stat,
                                const double* v, const double* F, const double* S, const double* P,
                                vsa_frame_result* recs, vsa_shot_result* shots, int32_t shots_cap,
                                int32_t* n_shots, int32_t* log, int32_t log_cap, int32_t* n_log, hipStream_t s) {
    hipLaunchKernelGGL(k_decide_replay, dim3(1), dim3(64), 0, s, sd, st, res, dp, T, act, swr, stat, v, F, S, P,
                       recs, shots, shots_cap, n_shots, log, log_cap, n_log);
    return hipGetLastError();
}

}  // namespace vsa
