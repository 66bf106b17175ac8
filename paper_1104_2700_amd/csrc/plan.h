// Device-side planning of a force sweep, shared by the standalone plan
// kernel and the fused block-step selection kernel, plus the fixed-order
// reduction of j-chunk partial sums.
#pragma once

#include "hermite_internal.h"

namespace hm {

// ---- wave-level primitives (every lane of the wave must call them) ----
// The partner's value in step O of a butterfly in which the lanes of each
// aligned group of 2 O combine their values (every lane ends with the
// group's result).  Within a 16-lane row the partner comes through a DPP
// lane move: quad permutes for O = 1, 2, then the half-row and row mirrors
// for O = 4, 8.  After the earlier steps all lanes of a quad (of a half-row)
// hold the same value, so the mirror partner gives bit for bit the xor
// partner's result (steps must run in ascending O).  Across rows (O = 16,
// 32) the value goes through ds_bpermute.
template <int O>
__device__ __forceinline__ int lane_partner_i32(int v)
{
    static_assert(O == 1 || O == 2 || O == 4 || O == 8, "DPP steps");
    constexpr int kCtrl = O == 1 ? 0xB1 : O == 2 ? 0x4E : O == 4 ? 0x141 : 0x140;
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}

template <int O>
__device__ __forceinline__ int32_t lane_xor(int32_t v)
{
    if constexpr (O >= 16) return __shfl_xor(v, O);
    else return lane_partner_i32<O>(v);
}

template <int O>
__device__ __forceinline__ int64_t lane_xor(int64_t v)
{
    if constexpr (O >= 16) {
        return __shfl_xor(v, O);
    } else {
        const int lo = lane_partner_i32<O>((int)v);
        const int hi = lane_partner_i32<O>((int)(v >> 32));
        return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
    }
}

template <int O>
__device__ __forceinline__ double lane_partner(double v)
{
    return __longlong_as_double((long long)lane_xor<O>((int64_t)__double_as_longlong(v)));
}

template <int O>
__device__ __forceinline__ float lane_partner(float v)
{
    return __int_as_float(lane_xor<O>((int32_t)__float_as_int(v)));
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v)
{
    v += lane_xor<1>(v);
    v += lane_xor<2>(v);
    v += lane_xor<4>(v);
    v += lane_xor<8>(v);
    v += lane_xor<16>(v);
    v += lane_xor<32>(v);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    v += lane_xor<1>(v);
    v += lane_xor<2>(v);
    v += lane_xor<4>(v);
    v += lane_xor<8>(v);
    v += lane_xor<16>(v);
    v += lane_xor<32>(v);
    return v;
}

__device__ __forceinline__ int64_t min_i64(int64_t a, int64_t b) { return b < a ? b : a; }

__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
    v = min_i64(v, lane_xor<1>(v));
    v = min_i64(v, lane_xor<2>(v));
    v = min_i64(v, lane_xor<4>(v));
    v = min_i64(v, lane_xor<8>(v));
    v = min_i64(v, lane_xor<16>(v));
    v = min_i64(v, lane_xor<32>(v));
    return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v)
{
    int32_t u;
    u = lane_xor<1>(v);  v = u > v ? u : v;
    u = lane_xor<2>(v);  v = u > v ? u : v;
    u = lane_xor<4>(v);  v = u > v ? u : v;
    u = lane_xor<8>(v);  v = u > v ? u : v;
    u = lane_xor<16>(v); v = u > v ? u : v;
    u = lane_xor<32>(v); v = u > v ? u : v;
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wave, by DPP lane moves:
// within each 16-lane row every lane adds the lanes 1, 2, 4 and 8 below it
// (zero past the row's start), then rows 1 and 3 add the last lane of the
// row below and rows 2 and 3 the last lane of row 1.
__device__ __forceinline__ int32_t wave_inscan(int32_t x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}


template <typename T>
__device__ inline int upper_bound_i64(const int64_t* a, int count, T key)
{
    int lo = 0, hi = count;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= (int64_t)key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int upper_bound_i32(const int32_t* a, int count, int key)
{
    int lo = 0, hi = count;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int lower_bound_i64(const int64_t* a, int count, int64_t key)
{
    int lo = 0, hi = count;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int lower_bound_idx(const int32_t* a, int count, int64_t key)
{
    int lo = 0, hi = count;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Counts a block step.  A step with no active particle is one past T_end
// (every live step has at least one): it leaves the counters untouched, so
// replaying extra steps after the end changes nothing.
__device__ inline void count_step(int64_t* counters, int64_t T, int32_t na)
{
    if (counters && na > 0) {
        // non-returning atomics: the caller does not wait for the update
        atomicAdd((unsigned long long*)&counters[0], 1ull);
        counters[3] = T;
        counters[4] = na;
        const int bin = 32 - __clz(na);                 // block-size histogram
        atomicAdd((unsigned long long*)&counters[kHistBase + bin], 1ull);
    }
}

// One workgroup selects the block of a system of n <= kFusedSelMax
// particles (procedure step 1): T = min_i (t_i + dt_i) into *T_out and the
// active indices, ascending, into s_idx (LDS).  Returns n_act, or 0 when
// T > T_end.  Each thread owns kFusedSelMax / kWG consecutive particles;
// their loads use clamped addresses so that all are in flight together.
// All threads call it.
__device__ inline int32_t select_in_lds(const int64_t* t, const int64_t* dt, int64_t n,
                                        int64_t T_end, int32_t* s_idx, int64_t* T_out)
{
    constexpr int kPer = kFusedSelMax / kWG;
    constexpr int kWaves = kWG / 64;
    __shared__ int64_t s_min[kWaves];
    __shared__ int32_t s_cnt[kWaves];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t base = (int64_t)tid * kPer;
    int64_t e[kPer];
    int64_t v = INT64_MAX;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t i = base + r;
        const int64_t ic = i < n ? i : n - 1;
        const int64_t x = t[ic] + dt[ic];
        e[r] = i < n ? x : INT64_MAX;
        v = e[r] < v ? e[r] : v;
    }
    v = wave_min_i64(v);
    if (lane == 0) s_min[wave] = v;
    __syncthreads();
    int64_t T = s_min[0];
    for (int w = 1; w < kWaves; ++w) T = s_min[w] < T ? s_min[w] : T;
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) c += e[r] == T ? 1 : 0;
    const int32_t x = wave_inscan(c);   // inclusive scan over the wave
    if (lane == 63) s_cnt[wave] = x;
    __syncthreads();
    int32_t pos = x - c, total = 0;
    for (int w = 0; w < kWaves; ++w) {
        pos += w < wave ? s_cnt[w] : 0;
        total += s_cnt[w];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r)
        if (e[r] == T) s_idx[pos++] = (int32_t)(base + r);
    __syncthreads();
    *T_out = T;
    return T <= T_end ? total : 0;
}

// ------------------------------------------------------------------------
// Plan: one workgroup (all kWG threads must call this) turns the active
// count into a split (lanes per particle L, chunk length jc) and a work
// list of (cluster, i-tile, j-chunk) items, and adds the sweep's
// interaction count to the counters.
// ------------------------------------------------------------------------
// Quotients of non-negative integers (b > 0).  The operands fit 32 bits in
// every plan of a realistic size, and the 32-bit division is a short
// sequence on the GPU, where a 64-bit one is a long software routine (a
// dozen of them made up most of a plan's latency).
__host__ __device__ inline int64_t div_floor(int64_t a, int64_t b)
{
    if ((((uint64_t)a | (uint64_t)b) >> 32) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}

__host__ __device__ inline int64_t div_ceil(int64_t a, int64_t b)
{
    const int64_t q = div_floor(a, b);
    return q * b != a ? q + 1 : q;
}

// ceil(a / b) for b a power of two (a shift), else div_ceil.
__host__ __device__ inline int64_t div_ceil_p2(int64_t a, int64_t b)
{
    if ((b & (b - 1)) == 0) return (a + b - 1) >> __builtin_ctzll((unsigned long long)b);
    return div_ceil(a, b);
}

// The split for na active particles of (at most) c_act active clusters:
// lanes per particle L, particles per item ti, chunk length jc.  (Also
// evaluated on the host, to size the grid of the fused select + sweep.)
__host__ __device__ inline void plan_split(const SweepArgs& a, int32_t na, int64_t c_act,
                                           int32_t* L_out, int32_t* ti_out, int64_t* jc_out)
{
    const int C = a.n_clusters;
    // Work items wanted (about one per resident workgroup slot, times the
    // tuning factor), and the most j-chunks a cluster can give (each chunk
    // at least one LDS tile, all partial sums in the buffer).
    const int64_t want = (int64_t)(a.target_lanes / kWG) > 0 ? a.target_lanes / kWG : 1;
    int64_t s_cap = a.one_chunk ? 1 : (a.n_cmax + kTJ - 1) / kTJ;
    if (na > 0) {
        const int64_t buf_cap = div_floor(a.partial_cap, kRows * (int64_t)na);
        if (buf_cap < s_cap) s_cap = buf_cap > 0 ? buf_cap : 1;
    }
    // Fewest lanes per particle that (a) still yields enough items and
    // (b) keeps tiles at least half full given the active particles per
    // active cluster: more particles per item means more work per staged j
    // tile, but a tile larger than a cluster's active run leaves lanes idle.
    const int64_t per_cluster = div_ceil(na, c_act);
    int32_t L = 1;
    for (; L < 64; L <<= 1) {
        const int64_t ti_l = (int64_t)a.ipl * (kWG / L);
        const int64_t tiles = div_ceil_p2(na, ti_l) + (C > 1 ? c_act : 0);
        if (tiles * s_cap >= want && ti_l <= 2 * per_cluster) break;
    }
    const int64_t ti_l = (int64_t)a.ipl * (kWG / L);
    const int64_t tiles = na > 0 ? div_ceil_p2(na, ti_l) + (C > 1 ? c_act : 0) : 1;
    int64_t S = div_ceil(want, tiles);
    if (S > s_cap) S = s_cap;
    if (S < 1) S = 1;
    int64_t jc = div_ceil(a.n_cmax, S);
    const int64_t jmin = (int64_t)L * a.min_j_per_lane;
    if (jc < jmin) jc = jmin;
    jc = (jc + kTJ - 1) / kTJ * kTJ;
    // rounding jc up can only lower the chunk count, so the buffer fits
    *L_out = L;
    *ti_out = (int32_t)ti_l;
    *jc_out = jc;
}

// The same split evaluated by a wave (lanes 0-6 at least must call it, with
// the same arguments): lane k takes the candidate L = 2^k, its tile count,
// chunk count and chunk length in parallel, a ballot picks the fewest lanes
// that satisfy both conditions (else 64) and that lane's chunk length is
// read back.  Every value is the one plan_split computes; only the serial
// search is gone.
__device__ inline void plan_split_wave(const SweepArgs& a, int32_t na, int64_t c_act,
                                       int32_t* L_out, int32_t* ti_out, int64_t* jc_out)
{
    const int C = a.n_clusters;
    const int64_t want = (int64_t)(a.target_lanes / kWG) > 0 ? a.target_lanes / kWG : 1;
    int64_t s_cap = a.one_chunk ? 1 : (a.n_cmax + kTJ - 1) / kTJ;
    if (na > 0) {
        const int64_t buf_cap = div_floor(a.partial_cap, kRows * (int64_t)na);
        if (buf_cap < s_cap) s_cap = buf_cap > 0 ? buf_cap : 1;
    }
    const int64_t per_cluster = div_ceil(na, c_act);
    const int lane = threadIdx.x & 63;
    const int k = lane < 7 ? lane : 6;
    const int32_t Lk = 1 << k;
    const int64_t ti_k = (int64_t)a.ipl * (kWG / Lk);
    const int64_t tiles_k = div_ceil_p2(na, ti_k) + (C > 1 ? c_act : 0);
    const bool ok = k < 6 && tiles_k * s_cap >= want && ti_k <= 2 * per_cluster;
    const unsigned long long m = __ballot(ok);
    const int lg = m ? __builtin_ctzll(m) : 6;
    const int64_t tiles = na > 0 ? tiles_k : 1;
    int64_t S = div_ceil(want, tiles);
    if (S > s_cap) S = s_cap;
    if (S < 1) S = 1;
    int64_t jc = div_ceil(a.n_cmax, S);
    const int64_t jmin = (int64_t)Lk * a.min_j_per_lane;
    if (jc < jmin) jc = jmin;
    jc = (jc + kTJ - 1) / kTJ * kTJ;
    const int lo = __builtin_amdgcn_readlane((int)jc, lg);
    const int hi = __builtin_amdgcn_readlane((int)(jc >> 32), lg);
    *L_out = 1 << lg;
    *ti_out = (int32_t)((int64_t)a.ipl * (kWG >> lg));
    *jc_out = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ inline int32_t block_exscan(int32_t v, int32_t* total)
{
    __shared__ int32_t s_w[kWG / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t x = wave_inscan(v);
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int32_t off = x - v, tot = 0;
    for (int w = 0; w < kWG / 64; ++w) {
        off += w < wave ? s_w[w] : 0;
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return off;
}

// One LDS round for three block-wide results (all kWG threads call it):
// the exclusive scan of v (returned; *total gets the sum), the sum of
// *sum and the maximum of *mx (both replaced by the block's).
__device__ inline int32_t block_exscan_sum_max(int32_t v, int32_t* total, int64_t* sum,
                                               int32_t* mx)
{
    __shared__ int32_t s_w[kWG / 64];
    __shared__ int64_t s_s[kWG / 64];
    __shared__ int32_t s_m[kWG / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t x = wave_inscan(v);
    int64_t sv = wave_sum_i64(*sum);
    int32_t m = wave_max_i32(*mx);
    if (lane == 63) {
        s_w[wave] = x;
        s_s[wave] = sv;
        s_m[wave] = m;
    }
    __syncthreads();
    int32_t off = x - v, tot = 0;
    sv = 0;
    m = s_m[0];
    for (int w = 0; w < kWG / 64; ++w) {
        off += w < wave ? s_w[w] : 0;
        tot += s_w[w];
        sv += s_s[w];
        m = s_m[w] > m ? s_m[w] : m;
    }
    __syncthreads();
    *total = tot;
    *sum = sv;
    *mx = m;
    return off;
}

// s_start / s_off (optional, LDS): every cluster's first active position
// (s_start[C] = na) and its particle range, as the ensemble selection has
// them at hand; without them the plan reads offsets and the selection's
// act_start from global memory, or searches idx.
__device__ inline void plan_body(const SweepArgs& a, int32_t na_in,
                                 const int32_t* s_start = nullptr, const int64_t* s_off = nullptr)
{
    const int tid = threadIdx.x;
    const int32_t na = na_in < 0 ? 0 : (na_in > a.n_act_max ? a.n_act_max : na_in);
    const int C = a.n_clusters;
    if (C == 1) {
        // one system: everything follows from na and n, no scans needed
        if (tid >= 64) return;
        int32_t L, ti;
        int64_t jc;
        plan_split_wave(a, na, 1, &L, &ti, &jc);
        if (tid == 0) {
            const int32_t tiles = (int32_t)div_ceil_p2(na, ti);
            const int32_t ch = na > 0 ? (int32_t)div_ceil(a.n, jc) : 0;
            a.act_start[0] = 0;
            a.act_cnt[0] = na;
            a.chunks[0] = ch;
            a.item_off[0] = 0;
            a.item_off[1] = tiles * ch;
            SweepPlan* P = a.plan;
            P->n_act = na;
            P->L = L;
            P->ti = ti;
            P->s_max = ch;
            P->jc = jc;
            P->total_items = tiles * ch;
            P->fp64_all = (a.fp64_inter_below > 0 && (int64_t)na * a.n < a.fp64_inter_below) ? 1 : 0;
            if (a.counters && na > 0)
                atomicAdd((unsigned long long*)&a.counters[1],
                          (unsigned long long)((int64_t)na * a.n));
        }
        return;
    }
    const int per = (C + kWG - 1) / kWG;
    const int c0 = tid * per;
    const int c1 = (c0 + per < C) ? c0 + per : C;

    // 1. the active run of every cluster (idx is ascending)
    int32_t nact_c = 0;
    for (int c = c0; c < c1; ++c) {
        const int64_t o0 = s_off ? s_off[c] : a.offsets[c];
        const int64_t o1 = s_off ? s_off[c + 1] : a.offsets[c + 1];
        int32_t st, cnt;
        if (s_start) {
            st = s_start[c];
            cnt = s_start[c + 1] - st;
        } else if (a.sel_clusters) {
            // starts recorded by the selection (only when it had active
            // particles); a cluster starting at n (empty, at the end) has
            // its run at na
            if (na == 0) {
                st = 0;
                cnt = 0;
            } else {
                st = o0 >= a.n ? na : a.act_start[c];
                const int32_t nx = (c + 1 < C && o1 < a.n) ? a.act_start[c + 1] : na;
                cnt = nx - st;
            }
            if (o0 >= a.n || na == 0) a.act_start[c] = st;
            a.act_cnt[c] = cnt;
            nact_c += cnt > 0 ? 1 : 0;
            continue;
        } else if (a.idx == nullptr) {
            const int64_t e = o1 < na ? o1 : na;
            st = (int32_t)o0;
            cnt = e > o0 ? (int32_t)(e - o0) : 0;
        } else {
            st = lower_bound_idx(a.idx, na, o0);
            cnt = lower_bound_idx(a.idx, na, o1) - st;
        }
        a.act_start[c] = st;
        a.act_cnt[c] = cnt;
        nact_c += cnt > 0 ? 1 : 0;
    }
    int32_t c_act;
    (void)block_exscan(nact_c, &c_act);

    // 2. the split: lanes per particle L and chunk length jc (every thread
    // evaluates it; it depends only on na, c_act and the arguments)
    int32_t L, ti;
    int64_t jc;
    plan_split_wave(a, na, c_act > 0 ? c_act : 1, &L, &ti, &jc);

    // 3. work items per cluster and their offsets (a thread's clusters'
    // item counts kept in registers when it owns at most kPlanPer of them)
    constexpr int kPlanPer = kLdsClusters / kWG;
    int32_t items_c[kPlanPer];
    int32_t local = 0, cmax = 0;
    int64_t inter = 0;
    for (int c = c0; c < c1; ++c) {
        const int64_t o0 = s_off ? s_off[c] : a.offsets[c];
        const int64_t o1 = s_off ? s_off[c + 1] : a.offsets[c + 1];
        const int32_t cnt = s_start ? s_start[c + 1] - s_start[c] : a.act_cnt[c];
        const int32_t tiles = (int32_t)div_ceil_p2(cnt, ti);
        const int32_t ch = cnt > 0 ? (int32_t)div_ceil(o1 - o0, jc) : 0;
        a.chunks[c] = ch;
        if (c - c0 < kPlanPer) items_c[c - c0] = tiles * ch;
        local += tiles * ch;
        cmax = ch > cmax ? ch : cmax;
        inter += (int64_t)cnt * (o1 - o0);
    }
    int32_t total;
    int32_t base = block_exscan_sum_max(local, &total, &inter, &cmax);
    for (int c = c0; c < c1; ++c) {
        a.item_off[c] = base;
        base += c - c0 < kPlanPer ? items_c[c - c0]
                                  : (int32_t)div_ceil_p2(a.act_cnt[c], ti) * a.chunks[c];
    }
    if (tid == 0) {
        a.item_off[C] = total;
        SweepPlan* P = a.plan;
        P->n_act = na;
        P->L = L;
        P->ti = ti;
        P->s_max = cmax;
        P->jc = jc;
        P->total_items = total;
        P->fp64_all = (a.fp64_inter_below > 0 && inter < a.fp64_inter_below) ? 1 : 0;
        if (a.counters && inter > 0)
            atomicAdd((unsigned long long*)&a.counters[1], (unsigned long long)inter);
    }
}

__device__ inline int cluster_of(const SweepArgs& a, int p)
{
    if (a.n_clusters <= 1) return 0;
    if (a.act_cluster) return a.act_cluster[p];
    const int i = a.idx ? a.idx[p] : p;
    return upper_bound_i64(a.offsets, a.n_clusters + 1, i) - 1;
}

// The sweep's error estimates travel as two FP32 numbers in the bits of
// one double (row 7 of the partial sums): the sums over the lane's FP32
// runs of |run sum|^2 for the acceleration (lo word) and the jerk (hi).
__device__ __forceinline__ double pack_est(float ea, float ej)
{
    const uint64_t b = (uint64_t)__float_as_uint(ea) | ((uint64_t)__float_as_uint(ej) << 32);
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ void unpack_est(double d, float* ea, float* ej)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    *ea = __uint_as_float((uint32_t)b);
    *ej = __uint_as_float((uint32_t)(b >> 32));
}

// Sum, in chunk order, of the partial results of active position p:
// out = acc xyz, jerk xyz, pot, and (row 7) the packed error estimates.
// One thread per particle.  Chunks are read kReduceBatch at a time from
// clamped addresses, so their loads are in flight together; the sum is
// still taken in chunk order (a chunk past the end adds +0.0, which leaves
// a sum that started at +0.0 unchanged bit for bit).
constexpr int kReduceBatch = 4;

// j-chunks of active position p (its cluster's).
__device__ inline int chunks_of(const SweepArgs& a, int p)
{
    return a.n_clusters <= 1 ? a.plan->s_max : a.chunks[cluster_of(a, p)];
}

__device__ inline void reduce_partials_ch(const SweepArgs& a, int na, int p, int ch,
                                          double out[kRows])
{
#pragma unroll
    for (int q = 0; q < kRows; ++q) out[q] = 0.0;
    float ea = 0.0f, ej = 0.0f;
    for (int k = 0; k < ch; k += kReduceBatch) {
        double v[kReduceBatch][kRows];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int kk = k + u < ch ? k + u : ch - 1;
#pragma unroll
            for (int q = 0; q < kRows; ++q)
                v[u][q] = a.partial[((int64_t)kk * kRows + q) * na + p];
        }
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
#pragma unroll
            for (int q = 0; q < kRows - 1; ++q) out[q] += k + u < ch ? v[u][q] : 0.0;
            float xa, xj;
            unpack_est(v[u][kRows - 1], &xa, &xj);
            ea += k + u < ch ? xa : 0.0f;
            ej += k + u < ch ? xj : 0.0f;
        }
    }
    out[kRows - 1] = pack_est(ea, ej);
}

template <int O>
__device__ __forceinline__ void wave_sum_step(double* out, float& ea, float& ej)
{
#pragma unroll
    for (int q = 0; q < kRows - 1; ++q) out[q] += lane_partner<O>(out[q]);
    ea += lane_partner<O>(ea);
    ej += lane_partner<O>(ej);
}

// The same sum by a whole wave (for many chunks): lane l adds chunks
// l, l + 64, ... in order, then a fixed xor butterfly combines the lanes.
// Every lane returns the total.  Deterministic for a given chunk count.
__device__ inline void reduce_partials(const SweepArgs& a, int na, int p, double out[kRows])
{
    reduce_partials_ch(a, na, p, chunks_of(a, p), out);
}

__device__ inline void reduce_partials_wave_ch(const SweepArgs& a, int na, int p, int ch,
                                               int lane, double out[kRows])
{
#pragma unroll
    for (int q = 0; q < kRows; ++q) out[q] = 0.0;
    float ea = 0.0f, ej = 0.0f;
    for (int k = lane; k < ch; k += 64) {
#pragma unroll
        for (int q = 0; q < kRows - 1; ++q) out[q] += a.partial[((int64_t)k * kRows + q) * na + p];
        float xa, xj;
        unpack_est(a.partial[((int64_t)k * kRows + kRows - 1) * na + p], &xa, &xj);
        ea += xa;
        ej += xj;
    }
    // every row takes each butterfly step together (independent reads
    // issued back to back)
    wave_sum_step<1>(out, ea, ej);
    wave_sum_step<2>(out, ea, ej);
    wave_sum_step<4>(out, ea, ej);
    wave_sum_step<8>(out, ea, ej);
    wave_sum_step<16>(out, ea, ej);
    wave_sum_step<32>(out, ea, ej);
    out[kRows - 1] = pack_est(ea, ej);
}

__device__ inline void reduce_partials_wave(const SweepArgs& a, int na, int p, int lane,
                                            double out[kRows])
{
    reduce_partials_wave_ch(a, na, p, chunks_of(a, p), lane, out);
}

// Position and velocity of particle i for the sweep: predicted on the fly
// (Taylor predictor, equations (xpred), (vpred), Horner form with FMA) or
// read from the predicted arrays.
__device__ inline void fetch_particle(const SweepArgs& a, int64_t i, int64_t T, double r[3],
                                      double w[3])
{
    const int64_t n = a.n;
    if (a.pred_x) {
        const double h = (double)(T - a.pred_t[i]) * a.tick;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t o = d * n + i;
            const double ac = a.pred_a[o], jk = a.pred_j[o];
            r[d] = fma(h, fma(h, fma(h, jk * (1.0 / 6.0), ac * 0.5), a.pred_v[o]), a.pred_x[o]);
            w[d] = fma(h, fma(h, jk * 0.5, ac), a.pred_v[o]);
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r[d] = a.xp[d * n + i];
            w[d] = a.vp[d * n + i];
        }
    }
}

// Chunk counts above kWaveReduceChunks use the wave-per-particle
// reduction, unless the active block is large enough that one thread per
// particle already fills the chip: then the thread form, whose loads are
// coalesced over particles, is the faster one.
constexpr int kWaveReduceChunks = 16;
constexpr int kThreadReduceMinAct = 16384;

__device__ __forceinline__ bool thread_reduce(int s_max, int na)
{
    return s_max <= kWaveReduceChunks || na >= kThreadReduceMinAct;
}

// ------------------------------------------------------------------------
// A-posteriori FP64 refinement of the mixed precisions.
//
// Each lane of a mixed sweep accumulates E = sum over its FP32 runs of
// |run sum|^2 (acceleration and jerk separately).  With the near pairs in
// FP64, a particle's remaining error is a random walk of per-term FP32
// errors, and u32 sqrt(E) tracks its size: the ratio of the true error to
// it stays below about 13 on the N = 65536 Plummer sample (CPU emulation
// of the kernel's arithmetic).  A particle whose u32 sqrt(E) exceeds
// kRefineRel times its acceleration or jerk magnitude could come near the
// 1e-6 bar (a sum that almost cancels).  The reduce stage flags such
// particles; its last workgroup lists them in active-list order and plans
// a second sweep, in FP64, with the flagged particles as its active list
// (j is streamed once per tile of them, as in any sweep); their refined
// sums then replace the mixed ones.
// ------------------------------------------------------------------------
constexpr double kRefineRel = 4e-8;

__device__ inline bool needs_refine(const SweepArgs& a, const double s[kRows])
{
    if (!a.refine) return false;
    float ea, ej;
    unpack_est(s[kRows - 1], &ea, &ej);
    const double u32 = 0x1p-24;
    const double A = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double J = sqrt(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    return u32 * sqrt((double)ea) > kRefineRel * A || u32 * sqrt((double)ej) > kRefineRel * J;
}

// Exclusive scan of one value per thread over the workgroup (all kWG
// threads call it); *total receives the sum.
// The flagging reduce handles the active positions in units: one round of
// a workgroup, kWG positions (a thread each) or kWG / 64 (a wave each).
// Every thread of the workgroup calls this once per round, with its flag
// (only for a position it owns): the unit's flagged positions are written
// compactly at the start of its own position range in ref_tmp and their
// count to ref_ucnt[unit].  ref_pos of every owned position becomes -1.
__device__ inline void flag_unit(const SweepArgs& a, int unit, int base, int p, bool owner,
                                 bool flag)
{
    int32_t tot;
    const int32_t off = block_exscan(owner && flag ? 1 : 0, &tot);
    if (owner) {
        a.ref_pos[p] = -1;
        if (flag) a.ref_tmp[base + off] = p;
    }
    if (threadIdx.x == 0) a.ref_ucnt[unit] = tot;
}

// One workgroup, after the flagging reduce: the refine list from the
// units' counts and compacted positions, in unit order (with clusters,
// grouped by cluster: each cluster's run starts at the sum of the counts
// before it, entries in any order within it), ref_pos of the flagged
// positions set to their slots, and the plan of the refine sweep ra.
// Returns the count.  Which slot a particle takes does not change its
// refined sums: every slot is swept with the same split.
__device__ inline int32_t build_refine_list(const SweepArgs& a, const SweepArgs& ra, int32_t na,
                                            int unit_size)
{
    __shared__ int32_t s_run;
    const int tid = threadIdx.x;
    const int nu = (na + unit_size - 1) / unit_size;
    // units' counts -> their first slot (exclusive scan, kWG units at a time)
    if (tid == 0) s_run = 0;
    __syncthreads();
    for (int u0 = 0; u0 < nu; u0 += kWG) {
        const int u = u0 + tid;
        const int32_t v = u < nu ? a.ref_ucnt[u] : 0;
        int32_t tot;
        const int32_t off = block_exscan(v, &tot);
        if (u < nu) a.ref_ucnt[u] = s_run + off;
        __syncthreads();
        if (tid == 0) s_run += tot;
        __syncthreads();
    }
    const int32_t cnt = s_run;
    const int C = a.n_clusters;
    if (C == 1) {
        for (int u = tid; u < nu; u += kWG) {
            const int32_t k0 = a.ref_ucnt[u];
            const int32_t k1 = u + 1 < nu ? a.ref_ucnt[u + 1] : cnt;
            for (int32_t k = k0; k < k1; ++k) {
                const int p = a.ref_tmp[u * unit_size + (k - k0)];
                a.ref_idx[k] = a.idx ? a.idx[p] : p;
                a.ref_p[k] = p;
                a.ref_pos[p] = k;
            }
        }
    } else {
        // per-cluster counts, their exclusive scan (the run starts of the
        // refine sweep) and placement through per-cluster cursors
        for (int c = tid; c < C; c += kWG) a.ref_ccnt[c] = 0;
        __syncthreads();
        for (int u = tid; u < nu; u += kWG) {
            const int32_t k0 = a.ref_ucnt[u];
            const int32_t k1 = u + 1 < nu ? a.ref_ucnt[u + 1] : cnt;
            for (int32_t k = k0; k < k1; ++k)
                atomicAdd(&a.ref_ccnt[cluster_of(a, a.ref_tmp[u * unit_size + (k - k0)])], 1);
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) s_run = 0;
        __syncthreads();
        for (int c0 = 0; c0 < C; c0 += kWG) {
            const int c = c0 + tid;
            const int32_t v = c < C ? a.ref_ccnt[c] : 0;
            int32_t tot;
            const int32_t off = block_exscan(v, &tot);
            if (c < C) {
                ra.act_start[c] = s_run + off;
                a.ref_ccnt[c] = s_run + off;
            }
            __syncthreads();
            if (tid == 0) s_run += tot;
            __syncthreads();
        }
        __threadfence_block();
        for (int u = tid; u < nu; u += kWG) {
            const int32_t k0 = a.ref_ucnt[u];
            const int32_t k1 = u + 1 < nu ? a.ref_ucnt[u + 1] : cnt;
            for (int32_t k = k0; k < k1; ++k) {
                const int p = a.ref_tmp[u * unit_size + (k - k0)];
                const int32_t slot = atomicAdd(&a.ref_ccnt[cluster_of(a, p)], 1);
                a.ref_idx[slot] = a.idx ? a.idx[p] : p;
                a.ref_p[slot] = p;
                a.ref_pos[p] = slot;
            }
        }
        __threadfence_block();
        __syncthreads();
    }
    plan_body(ra, cnt);
    return cnt;
}

}  // namespace hm
