// O(N) and O(N_act) stages of a block step on gfx950: block selection,
// predictor, corrector + next timestep, first timestep, energy sums.
// All are memory/latency bound; every thread handles whole particles and
// reads/writes SoA arrays with unit stride.
#include "hermite_internal.h"
#include "plan.h"

namespace hm {
namespace {

constexpr int kSelPer = 16;                // particles per thread in select
constexpr int kSelBlock = kWG * kSelPer;   // particles per select block

// ---- block selection (procedure step 1) ---------------------------------
// t_i + dt_i of particle i, or INT64_MAX past the end (n >= 1).  The load
// address is clamped rather than guarded, so a thread issues all of its
// loads before it waits for any: a guarded load compiles to a branch that
// waits for each element in turn.
__device__ __forceinline__ int64_t next_time(const int64_t* t, const int64_t* dt, int64_t n,
                                             int64_t i)
{
    const int64_t ic = i < n ? i : n - 1;
    const int64_t e = t[ic] + dt[ic];
    return i < n ? e : INT64_MAX;
}

// Block-wide (kWG threads) minimum / sum / exclusive scan by wave shuffles
// and one round through LDS (s: kWG/64 entries); every thread calls and
// every thread gets the result.  A tree through LDS would take two barriers
// per level.
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* s)
{
    v = wave_min_i64(v);
    __syncthreads();                     // s may still be read by a previous call
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = s[0];
    for (int w = 1; w < kWG / 64; ++w) r = s[w] < r ? s[w] : r;
    return r;
}

__device__ __forceinline__ int32_t block_sum_i32(int32_t v, int32_t* s)
{
    v = wave_sum_i32(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t r = 0;
    for (int w = 0; w < kWG / 64; ++w) r += s[w];
    return r;
}

// Exclusive prefix of v over the block's threads; *total gets the sum.
__device__ __forceinline__ int32_t block_exscan_i32(int32_t v, int32_t* s, int32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t x = wave_inscan(v);
    __syncthreads();
    if (lane == 63) s[wave] = x;
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int w = 0; w < kWG / 64; ++w) {
        off += w < wave ? s[w] : 0;
        tot += s[w];
    }
    *total = tot;
    return off + x - v;
}

// Stage 1: per-block minimum of t_i + dt_i.
__global__ void __launch_bounds__(kWG) sel_min_kernel(int64_t n, const int64_t* t,
                                                      const int64_t* dt,
                                                      int64_t* block_min)
{
    __shared__ int64_t sh[kWG / 64];
    const int64_t base = (int64_t)blockIdx.x * kSelBlock;
    int64_t v = INT64_MAX;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        const int64_t e = next_time(t, dt, n, base + (int64_t)r * kWG + threadIdx.x);
        v = e < v ? e : v;
    }
    const int64_t bmin = block_min_i64(v, sh);
    if (threadIdx.x == 0) block_min[blockIdx.x] = bmin;
}

__device__ int64_t block_min_all(const int64_t* block_min, int nb, int64_t* sh)
{
    int64_t v = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kWG) v = block_min[b] < v ? block_min[b] : v;
    return block_min_i64(v, sh);
}

// Stage 2: T from all block minima; count the active particles per block.
__global__ void __launch_bounds__(kWG) sel_count_kernel(int64_t n, const int64_t* t,
                                                        const int64_t* dt,
                                                        const int64_t* block_min,
                                                        int nb, int32_t* block_cnt,
                                                        int64_t* T_out)
{
    __shared__ int64_t sh[kWG];
    __shared__ int32_t shc[kWG];
    const int64_t T = block_min_all(block_min, nb, sh);
    const int64_t base = (int64_t)blockIdx.x * kSelBlock;
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r)
        c += next_time(t, dt, n, base + (int64_t)r * kWG + threadIdx.x) == T ? 1 : 0;
    const int32_t bcnt = block_sum_i32(c, shc);
    if (threadIdx.x == 0) {
        block_cnt[blockIdx.x] = bcnt;
        if (blockIdx.x == 0) *T_out = T;
    }
}

// Stages 1 and 2 in one launch (block-step path): every block finds its
// minimum of t_i + dt_i and how many of its particles attain it; the last
// block to finish (atomic ticket) takes the global minimum T and keeps the
// counts of the blocks whose minimum is T.
__global__ void __launch_bounds__(kWG) sel_min_count_kernel(int64_t n, const int64_t* t,
                                                            const int64_t* dt,
                                                            int64_t* block_min,
                                                            int32_t* block_cnt, int nb,
                                                            int64_t* T_out, uint32_t* ticket)
{
    __shared__ int64_t sh[kWG];
    __shared__ int32_t shc[kWG];
    __shared__ int32_t s_last;
    const int64_t base = (int64_t)blockIdx.x * kSelBlock;
    int64_t e[kSelPer];
    int64_t v = INT64_MAX;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        e[r] = next_time(t, dt, n, base + (int64_t)r * kWG + threadIdx.x);
        v = e[r] < v ? e[r] : v;
    }
    const int64_t bmin = block_min_i64(v, sh);
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) c += (e[r] == bmin) ? 1 : 0;
    const int32_t bcnt = block_sum_i32(c, shc);
    if (threadIdx.x == 0) {
        block_min[blockIdx.x] = bmin;
        block_cnt[blockIdx.x] = bcnt;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(ticket, 1u) == (uint32_t)(nb - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int64_t T = block_min_all(block_min, nb, sh);
    for (int b = threadIdx.x; b < nb; b += kWG)
        if (block_min[b] != T) block_cnt[b] = 0;
    if (threadIdx.x == 0) {
        *T_out = T;
        *ticket = 0u;
    }
}

// Stage 3: each block's output offset is the sum of the counts before it;
// a block-wide scan places every active index in ascending order.  The
// block-step path also predicts the block's particles here (T is known),
// and the last block to finish (atomic ticket) totals n_act, updates the
// counters and builds the sweep plan, so that one launch does the work of
// three.
struct PredictArgs {
    double tick;
    const double* x;
    const double* v;
    const double* a;
    const double* j;
    double* xp;
    double* vp;
};

__device__ __forceinline__ void predict_one(int64_t n, int64_t i, int64_t T, const int64_t* t,
                                            const PredictArgs& pa)
{
    const double h = (double)(T - t[i]) * pa.tick;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t o = d * n + i;
        const double a2 = pa.a[o] * 0.5;
        const double j6 = pa.j[o] * (1.0 / 6.0);
        const double j2 = pa.j[o] * 0.5;
        pa.xp[o] = fma(h, fma(h, fma(h, j6, a2), pa.v[o]), pa.x[o]);
        pa.vp[o] = fma(h, fma(h, j2, pa.a[o]), pa.v[o]);
    }
}

// Writes the active indices of elements i = base .. base+kSelPer-1 from
// position pos on (f: which are active).  With clusters (cl_off = the C
// cluster starts, in LDS or global memory) it also records, for every
// cluster that starts in this range, how many active particles precede
// that start (act_start), and the cluster of every active position
// (act_cluster): the plan and the reduction then need no searches.
__device__ __forceinline__ void write_active(int64_t n, int64_t base, const bool* f, int32_t pos,
                                             int32_t* idx, const int64_t* cl_off, int C,
                                             int32_t* act_start, int32_t* act_cluster)
{
    if (!cl_off) {
        for (int r = 0; r < kSelPer; ++r)
            if (f[r]) idx[pos++] = (int32_t)(base + r);
        return;
    }
    int cn = lower_bound_i64(cl_off, C, base);   // first cluster starting at >= base
    for (int r = 0; r < kSelPer; ++r) {
        const int64_t i = base + r;
        if (i >= n) break;
        while (cn < C && cl_off[cn] == i) act_start[cn++] = pos;
        if (f[r]) {
            idx[pos] = (int32_t)i;
            act_cluster[pos] = cn - 1;
            ++pos;
        }
    }
}

// Stages the C cluster starts in LDS when they fit (all threads call);
// returns the table to search.
__device__ __forceinline__ const int64_t* stage_cluster_starts(const SweepArgs& sa, int64_t* s_off)
{
    if (!sa.sel_clusters || sa.n_clusters <= 1) return nullptr;
    const int C = sa.n_clusters;
    if (C > kLdsClusters) return sa.offsets;
    for (int k = threadIdx.x; k < C; k += kWG) s_off[k] = sa.offsets[k];
    __syncthreads();
    return s_off;
}

// Writes this block's active indices; returns the block's active count.
__device__ int32_t sel_write_body(int64_t n, const int64_t* t, const int64_t* dt,
                                  const int32_t* block_cnt, int64_t T, bool live,
                                  int32_t* idx, int32_t* sh, const int64_t* cl_off = nullptr,
                                  int C = 1, int32_t* act_start = nullptr,
                                  int32_t* act_cluster = nullptr)
{
    // this thread's particles are base + tid*kSelPer + r (contiguous per
    // thread so that a scan over threads keeps ascending order)
    const int64_t base = (int64_t)blockIdx.x * kSelBlock + (int64_t)threadIdx.x * kSelPer;
    bool f[kSelPer];
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        f[r] = next_time(t, dt, n, base + r) == T;
        c += f[r] ? 1 : 0;
    }
    int32_t pre = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kWG) pre += block_cnt[b];
    const int32_t off = block_sum_i32(pre, sh);
    int32_t block_total;
    const int32_t pos = off + block_exscan_i32(c, sh + kWG / 64, &block_total);
    if (live) write_active(n, base, f, pos, idx, cl_off, C, act_start, act_cluster);
    __syncthreads();
    return off + block_total;
}

__global__ void __launch_bounds__(kWG) sel_write_kernel(int64_t n, const int64_t* t,
                                                        const int64_t* dt,
                                                        const int32_t* block_cnt,
                                                        int nb, const int64_t* T_in,
                                                        int64_t T_end, int32_t* idx,
                                                        int32_t* n_act,
                                                        int64_t* counters)
{
    __shared__ int32_t sh[kWG];
    const int64_t T = *T_in;
    const bool live = T <= T_end;
    const int32_t upto = sel_write_body(n, t, dt, block_cnt, T, live, idx, sh);
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) {
        const int32_t na = live ? upto : 0;
        *n_act = na;
        count_step(counters, T, na);
    }
}

__global__ void __launch_bounds__(kWG) sel_write_plan_kernel(
    int64_t n, const int64_t* t, const int64_t* dt, const int32_t* block_cnt, int nb,
    const int64_t* T_in, int64_t T_end, int32_t* idx, int32_t* n_act, int64_t* counters,
    SweepArgs sa, uint32_t* ticket)
{
    __shared__ int32_t sh[kWG];
    __shared__ int32_t s_last;
    __shared__ int32_t s_na;
    __shared__ int64_t s_off[kLdsClusters];
    const int64_t* cl_off = stage_cluster_starts(sa, s_off);
    const int64_t T = *T_in;
    const bool live = T <= T_end;
    (void)sel_write_body(n, t, dt, block_cnt, T, live, idx, sh, cl_off, sa.n_clusters,
                         sa.act_start, sa.act_cluster);
    // the last block to arrive sees every block's indices
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(ticket, 1u) == (uint32_t)(nb - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    int32_t part = 0;
    for (int b = threadIdx.x; b < nb; b += kWG) part += block_cnt[b];
    const int32_t total = block_sum_i32(part, sh);
    if (threadIdx.x == 0) {
        const int32_t na = live ? total : 0;
        *n_act = na;
        count_step(counters, T, na);
        *ticket = 0u;
        s_na = na;
    }
    __syncthreads();
    plan_body(sa, s_na);
}

// The same list without the ticket, for many blocks: a last-block ticket
// costs a device-scope fence per block (about 65 ns each on this GPU, 0.26
// ms at 4096 blocks), a launch about 3 us.  Every block places its entries
// from the counts of the blocks before it, the last one publishes n_act,
// and sel_plan_kernel plans.
constexpr int kSelTicketMax = 48;   // selection blocks up to which the ticket is used

__global__ void __launch_bounds__(kWG) sel_write_list_kernel(
    int64_t n, const int64_t* t, const int64_t* dt, const int32_t* block_cnt, int nb,
    const int64_t* T_in, int64_t T_end, int32_t* idx, int32_t* n_act, int64_t* counters,
    SweepArgs sa)
{
    __shared__ int32_t sh[kWG];
    __shared__ int64_t s_off[kLdsClusters];
    const int64_t* cl_off = stage_cluster_starts(sa, s_off);
    const int64_t T = *T_in;
    const bool live = T <= T_end;
    const int32_t upto = sel_write_body(n, t, dt, block_cnt, T, live, idx, sh, cl_off,
                                        sa.n_clusters, sa.act_start, sa.act_cluster);
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) {
        const int32_t na = live ? upto : 0;
        *n_act = na;
        count_step(counters, T, na);
    }
}

__global__ void __launch_bounds__(kWG) sel_plan_kernel(SweepArgs sa, const int32_t* n_act)
{
    plan_body(sa, *n_act);
}

// Stages 1-3 and the sweep plan in one workgroup, for systems that fit one
// selection block (n <= kSelBlock): no cross-block ticket or fence, one
// launch instead of two.  Each thread owns kSelPer consecutive particles,
// so a scan over threads writes the active list in ascending order.
__global__ void __launch_bounds__(kWG) sel_single_plan_kernel(
    int64_t n, const int64_t* t, const int64_t* dt, int64_t T_end, int32_t* idx,
    int32_t* n_act, int64_t* T_out, int64_t* counters, SweepArgs sa)
{
    constexpr int kWaves = kWG / 64;
    __shared__ int64_t s_min[kWaves];
    __shared__ int32_t s_cnt[kWaves];
    __shared__ int64_t s_off[kLdsClusters];
    const int64_t* cl_off = stage_cluster_starts(sa, s_off);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t base = (int64_t)tid * kSelPer;
    int64_t e[kSelPer];
    int64_t v = INT64_MAX;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        e[r] = next_time(t, dt, n, base + r);
        v = e[r] < v ? e[r] : v;
    }
    // block minimum: wave butterfly, then the kWaves wave minima
    v = wave_min_i64(v);
    if (lane == 0) s_min[wave] = v;
    __syncthreads();
    int64_t T = s_min[0];
    for (int w = 1; w < kWaves; ++w) T = s_min[w] < T ? s_min[w] : T;
    const bool live = T <= T_end;
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) c += (e[r] == T) ? 1 : 0;
    // ascending positions: inclusive wave scan, then the wave offsets
    const int32_t x = wave_inscan(c);
    if (lane == 63) s_cnt[wave] = x;
    __syncthreads();
    int32_t off = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
        off += w < wave ? s_cnt[w] : 0;
        total += s_cnt[w];
    }
    if (live) {
        bool f[kSelPer];
#pragma unroll
        for (int r = 0; r < kSelPer; ++r) f[r] = e[r] == T;
        write_active(n, base, f, off + x - c, idx, cl_off, sa.n_clusters, sa.act_start,
                     sa.act_cluster);
    }
    __syncthreads();   // act_start complete before the plan reads it
    const int32_t na = live ? total : 0;
    if (tid == 0) {
        *T_out = T;
        *n_act = na;
        count_step(counters, T, na);
    }
    plan_body(sa, na);
}

// ---- block selection from the step-size order (procedure step 1) ---------
__device__ __forceinline__ int log2_step(int64_t dt)
{
    return 63 - __clzll((unsigned long long)dt);
}

// Step counts of the state and its consistency: every dt_i a power of two
// no finer than dt_floor, t_i >= 0 a multiple of dt_i, and (checked on the
// host) max t < min (t + dt).
__global__ void __launch_bounds__(kWG) level_count_kernel(LevelArgs L)
{
    __shared__ int32_t h[64];
    __shared__ int64_t s1[kWG / 64];
    __shared__ int32_t s2[kWG / 64];
    const int tid = threadIdx.x;
    if (tid < 64) h[tid] = 0;
    __syncthreads();
    int64_t tmax = INT64_MIN, nmin = INT64_MAX;
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + tid; i < L.n; i += (int64_t)gridDim.x * kWG) {
        const int64_t ti = L.t[i], di = L.dt[i];
        if (di < L.dt_floor || (di & (di - 1)) != 0 || ti < 0 || (ti & (di - 1)) != 0 ||
            ti > INT64_MAX - di) {
            bad = 1;
        } else {
            atomicAdd(&h[log2_step(di)], 1);
            nmin = ti + di < nmin ? ti + di : nmin;
        }
        tmax = ti > tmax ? ti : tmax;
    }
    nmin = block_min_i64(nmin, s1);
    tmax = ~block_min_i64(~tmax, s1);            // ~ reverses the order without overflow
    bad = block_sum_i32(bad, s2);
    if (tid == 0) {
        __hip_atomic_fetch_max(&L.misc[1], tmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_min(&L.misc[2], nmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bad) __hip_atomic_fetch_max(&L.misc[3], (int64_t)1, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid < 64 && h[tid] > 0) atomicAdd(&L.cnt[tid], h[tid]);
}

// Orders the particles by step size (a counting sort; the order within one
// step size is unspecified).
__global__ void __launch_bounds__(kWG) level_build_kernel(LevelArgs L)
{
    __shared__ int32_t h[64], base[64];
    const int tid = threadIdx.x;
    if (tid < 64) h[tid] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kWG + tid; i < L.n; i += (int64_t)gridDim.x * kWG)
        atomicAdd(&h[log2_step(L.dt[i])], 1);
    __syncthreads();
    if (tid < 64) {
        // this block's place in every step size: the sizes before it, then
        // the blocks that claimed that size before it
        const int32_t c = L.cnt[tid];
        const int32_t x = wave_inscan(c);
        const int32_t mine = h[tid];
        base[tid] = x - c + (mine > 0 ? atomicAdd(&L.cursor[tid], mine) : 0);
        h[tid] = 0;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kWG + tid; i < L.n; i += (int64_t)gridDim.x * kWG) {
        const int b = log2_step(L.dt[i]);
        L.perm[base[b] + atomicAdd(&h[b], 1)] = (int32_t)i;
    }
    if (blockIdx.x == 0 && tid == 0) {
        L.misc[0] = L.misc[1];
        *L.na = 0;
        *L.na_prev = 0;
    }
}

constexpr int kLevelLds = 2048;   // blocks re-sorted in LDS
constexpr int kLevelBatch = 8;    // elements per thread whose loads are issued together
constexpr int kLevelOrder = 4096; // one system: blocks listed in particle order
constexpr int kSelectGrid = 256;  // ensembles: workgroups of the selection

// Particle ids of positions p = p0 + u kWG + tid (u < kLevelBatch) of
// src[0, cnt) and, with_steps, their step sizes (log2), from lv[p] when
// given (the corrector's record, read in position order) else from dt of
// the id: every load is issued before any is used (addresses clamped to
// the last position, so none is conditional).
__device__ __forceinline__ void level_batch(const int32_t* src, const int64_t* dt, int32_t cnt,
                                            int32_t p0, int32_t (&id)[kLevelBatch],
                                            int (&b)[kLevelBatch], bool with_steps,
                                            const uint8_t* lv = nullptr)
{
#pragma unroll
    for (int u = 0; u < kLevelBatch; ++u) {
        const int32_t p = p0 + u * kWG + (int32_t)threadIdx.x;
        id[u] = src[p < cnt ? p : cnt - 1];
        if (with_steps && lv) b[u] = lv[p < cnt ? p : cnt - 1];
    }
    if (with_steps && !lv) {
        int64_t d[kLevelBatch];
#pragma unroll
        for (int u = 0; u < kLevelBatch; ++u) d[u] = dt[id[u]];
#pragma unroll
        for (int u = 0; u < kLevelBatch; ++u) b[u] = log2_step(d[u]);
    }
}

// out[pos] = v when 0 <= pos < cnt; otherwise records the inconsistency in
// misc[4] (reported by hermite_run) instead of writing out of range.
__device__ __forceinline__ bool level_put(const LevelArgs& L, int32_t* out, int32_t pos,
                                          int32_t cnt, int32_t v)
{
    if (pos >= 0 && pos < cnt) {
        out[pos] = v;
        return true;
    }
    __hip_atomic_store(&L.misc[4], (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int32_t wave_inscan_i32(int32_t x)
{
    return wave_inscan(x);
}

struct LevelLds {
    int32_t hist[64], cur[64], cnt[64];
    int32_t id[kLevelLds];
    int32_t aux[kLevelLds];
    uint8_t lv[kLevelLds];
};

// Re-sorts the last block, perm[0, m), by the steps the corrector gave it
// (a counting sort by step size; staged in LDS up to kLevelLds, else
// through tmp[0, m)); lv (or null: dt through perm) holds the new steps'
// log2 by position.  Every particle of that block had a step dividing
// the block time 2^z * odd and got a new one that divides it, and every
// particle after it has a larger step, so the whole order stays sorted.
// S.cnt (the order's step counts) gets the block's counts for steps <= 2^z.
// All threads of the workgroup call it; it ends with a barrier.
__device__ void level_resort(const LevelArgs& L, int32_t* perm, int32_t* tmp, int32_t m, int z,
                             LevelLds& S, const uint8_t* lv)
{
    const int tid = threadIdx.x;
    constexpr int kStride = kWG * kLevelBatch;
    const bool lds = m <= kLevelLds;
    if (tid < 64) S.hist[tid] = 0;
    __syncthreads();
    for (int32_t p0 = 0; p0 < m; p0 += kStride) {
        int32_t id[kLevelBatch];
        int b[kLevelBatch];
        level_batch(perm, L.dt, m, p0, id, b, true, lv);
#pragma unroll
        for (int u = 0; u < kLevelBatch; ++u) {
            const int32_t p = p0 + u * kWG + tid;
            if (p < m) {
                if (lds) {
                    S.id[p] = id[u];
                    S.lv[p] = (uint8_t)b[u];
                }
                atomicAdd(&S.hist[b[u]], 1);
            }
        }
    }
    __syncthreads();
    if (tid < 64) {
        const int32_t hb = S.hist[tid];
        S.cnt[tid] = (tid <= z ? 0 : S.cnt[tid]) + hb;
        S.cur[tid] = wave_inscan_i32(hb) - hb;
    }
    __syncthreads();
    if (lds) {
        for (int32_t p = tid; p < m; p += kWG)
            level_put(L, S.aux, atomicAdd(&S.cur[S.lv[p]], 1), m, S.id[p]);
        __syncthreads();
        for (int32_t p = tid; p < m; p += kWG) perm[p] = S.aux[p];
    } else {
        for (int32_t p0 = 0; p0 < m; p0 += kStride) {
            int32_t id[kLevelBatch];
            int b[kLevelBatch];
            level_batch(perm, L.dt, m, p0, id, b, true, lv);
#pragma unroll
            for (int u = 0; u < kLevelBatch; ++u)
                if (p0 + u * kWG + tid < m)
                    level_put(L, tmp, atomicAdd(&S.cur[b[u]], 1), m, id[u]);
        }
        __syncthreads();
        for (int32_t p0 = 0; p0 < m; p0 += kStride) {
            int32_t id[kLevelBatch];
            int b[kLevelBatch];
            level_batch(tmp, L.dt, m, p0, id, b, false);
#pragma unroll
            for (int u = 0; u < kLevelBatch; ++u) {
                const int32_t p = p0 + u * kWG + tid;
                if (p < m) perm[p] = id[u];
            }
        }
    }
    __syncthreads();
}

// The next block from the step counts (one lane per step size b, lanes of
// one wave): every particle's next time is the first multiple of its step
// after T_last, so the block time is the first multiple of the smallest
// occupied step, and the block is every particle whose step divides it.
// Returns the block time; *na its size (0 past T_end).
__device__ __forceinline__ int64_t level_next(int32_t cnt_b, int64_t Tlast, int64_t T_end,
                                              int32_t* na)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long occ = __ballot(cnt_b > 0);
    int64_t Tn = INT64_MAX;
    int32_t v = 0;
    if (occ != 0ull) {
        const int bmin = __builtin_ctzll(occ);
        Tn = ((Tlast >> bmin) + 1) << bmin;
        const int zn = __builtin_ctzll((unsigned long long)Tn);
        v = wave_sum_i32(lane <= zn ? cnt_b : 0);
    }
    *na = Tn > T_end ? 0 : v;
    return Tn;
}

// One system, one workgroup: the previous block re-sorted, the next block
// taken as the order's prefix (blocks above kLevelOrder are rewritten in
// ascending particle order, so that a wave's particles lie close together
// and fewer j-tiles need the self-pair mask), and the sweep planned.
__global__ void __launch_bounds__(kWG) level_select_kernel(LevelArgs L, SweepArgs sa)
{
    __shared__ LevelLds S;
    __shared__ int32_t s_scan[kWG / 64];
    __shared__ int32_t s_na;
    const int tid = threadIdx.x;
    const int32_t na_prev = *L.na_prev;
    int64_t Tlast = L.misc[0];
    if (tid < 64) S.cnt[tid] = L.cnt[tid];
    if (na_prev > 0) {
        Tlast = *L.T;
        level_resort(L, L.perm, L.tmp, na_prev, __builtin_ctzll((unsigned long long)Tlast), S,
                     L.lv);
        if (tid < 64) L.cnt[tid] = S.cnt[tid];
        if (tid == 0) L.misc[0] = Tlast;
    } else {
        __syncthreads();
    }
    if (tid < 64) {
        int32_t na;
        const int64_t Tn = level_next(S.cnt[tid], Tlast, L.T_end, &na);
        if (tid == 0) {
            s_na = na;
            *L.T = Tn;
            *L.na = na;
            count_step(L.counters, Tn, na);
        }
    }
    __syncthreads();
    const int32_t na = s_na;
    if (na <= kLevelOrder) {
        plan_body(sa, na);
        return;
    }
    // a large block: ascending particle order through a bitmap of the active
    // particles, written over the prefix of the order (its order within the
    // prefix is free: the next re-sort reorders it)
    constexpr int kStride = kWG * kLevelBatch;
    for (int32_t p0 = 0; p0 < na; p0 += kStride) {
        int32_t id[kLevelBatch];
        int b[kLevelBatch];
        level_batch(L.perm, L.dt, na, p0, id, b, false);
#pragma unroll
        for (int u = 0; u < kLevelBatch; ++u)
            if (p0 + u * kWG + tid < na) atomicOr(&L.bits[id[u] >> 5], 1u << (id[u] & 31));
    }
    __syncthreads();
    // thread t owns a contiguous run [wa, wb) of the bitmap's words
    const int64_t nw = (L.n + 31) >> 5;
    const int64_t tper = (nw + kWG - 1) / kWG;
    const int64_t wa = tid * tper < nw ? tid * tper : nw;
    const int64_t wb = wa + tper < nw ? wa + tper : nw;
    int32_t cnt = 0;
    for (int64_t w = wa; w < wb; ++w) cnt += __popc(L.bits[w]);
    int32_t total;
    int32_t pos = block_exscan_i32(cnt, s_scan, &total);
    for (int64_t w = wa; w < wb; ++w) {
        uint32_t word = L.bits[w];
        L.bits[w] = 0u;
        while (word) {
            level_put(L, L.perm, pos++, na, (int32_t)((w << 5) + __builtin_ctz(word)));
            word &= word - 1u;
        }
    }
    __syncthreads();
    plan_body(sa, na);
}

// Ensembles.  Cluster c keeps its own step-size order in its range of perm,
// perm[off_c, off_c+1), with its step counts ccnt[c][b] and their running
// sums ccum[c][b]; cnt[b] holds the counts of the whole ensemble.  All
// clusters share the block time, and cluster c's part of a block is a
// prefix of its range.

// Builds every cluster's order from t and dt (one workgroup per cluster).
__global__ void __launch_bounds__(kWG) cl_build_kernel(LevelArgs L)
{
    __shared__ int32_t h[64], base[64];
    const int tid = threadIdx.x, c = blockIdx.x;
    const int64_t o0 = L.offsets[c], o1 = L.offsets[c + 1];
    if (tid < 64) h[tid] = 0;
    __syncthreads();
    for (int64_t i = o0 + tid; i < o1; i += kWG) atomicAdd(&h[log2_step(L.dt[i])], 1);
    __syncthreads();
    if (tid < 64) {
        const int32_t k = h[tid];
        const int32_t x = wave_inscan_i32(k);
        base[tid] = x - k;
        L.ccnt[c * 64 + tid] = k;
        L.ccum[c * 64 + tid] = x;
        if (tid == 0) {
            L.cna[c] = 0;
            L.cst[c] = 0;
        }
    }
    __syncthreads();
    for (int64_t i = o0 + tid; i < o1; i += kWG) {
        const int b = log2_step(L.dt[i]);
        L.perm[o0 + atomicAdd(&base[b], 1)] = (int32_t)i;
    }
    if (c == 0 && tid == 0) {
        L.misc[0] = L.misc[1];
        *L.na = 0;
        *L.na_prev = 0;
    }
}

// Re-sorts every cluster's part of the last block by its new steps: one
// workgroup per cluster, each on its own range; the ensemble's counts take
// each cluster's changes (integer atomics, so their sum is exact).
__global__ void __launch_bounds__(kWG) cl_resort_kernel(LevelArgs L)
{
    __shared__ LevelLds S;
    const int tid = threadIdx.x, c = blockIdx.x;
    // every load this workgroup may need is issued before any is waited on
    const int32_t na_prev = *L.na_prev;
    const int64_t T_prev = *L.T;
    const int32_t m = L.cna[c];
    const int32_t pst = L.cst[c];
    const int64_t o = L.offsets[c], o1 = L.offsets[c + 1];
    const int32_t old = tid < 64 ? L.ccnt[c * 64 + tid] : 0;
    if (na_prev <= 0) return;
    if (c == 0 && tid == 0) L.misc[0] = T_prev;
    if (m <= 0) return;
    if ((int64_t)m > o1 - o || pst < 0 || (int64_t)pst + m > L.n) {
        if (tid == 0)
            __hip_atomic_store(&L.misc[4], (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (tid < 64) S.cnt[tid] = old;
    level_resort(L, L.perm + o, L.tmp + o, m, __builtin_ctzll((unsigned long long)T_prev), S,
                 L.lv ? L.lv + pst : nullptr);
    if (tid < 64) {
        const int32_t k = S.cnt[tid];
        L.ccnt[c * 64 + tid] = k;
        L.ccum[c * 64 + tid] = wave_inscan_i32(k);
        if (k != old) atomicAdd(&L.cnt[tid], k - old);
    }
}

// Selects the next block of an ensemble and lists it grouped by cluster.
// Every workgroup derives the block time and every cluster's count from
// the same tables (nothing here writes them), lists the blocks of clusters
// g, g + G, ... and records their sizes for the next re-sort; workgroup 0
// publishes the block time, n_act and the sweep plan (from the starts and
// ranges it holds in LDS, so the plan waits on no global load).
__global__ void __launch_bounds__(kWG) cl_select_kernel(LevelArgs L, SweepArgs sa)
{
    __shared__ int32_t s_start[kLdsClusters + 1];
    __shared__ int64_t s_off[kLdsClusters + 1];
    __shared__ int32_t s_scan[kWG / 64];
    __shared__ int32_t s_bm;
    const int tid = threadIdx.x, G = gridDim.x, g = blockIdx.x;
    const int C = L.n_clusters;
    // the loads that do not depend on each other, issued together: the
    // first kWG entries of this workgroup's first cluster's order among
    // them (most blocks take fewer)
    const int64_t Tlast = L.misc[0];
    const int32_t cnt_b = tid < 64 ? L.cnt[tid] : 0;
    int32_t pre = 0;
    if (g < C) {
        const int64_t o = L.offsets[g];
        if (o + tid < L.offsets[g + 1]) pre = L.perm[o + tid];
    }
    for (int c = tid; c <= C; c += kWG) s_off[c] = L.offsets[c];
    // the smallest occupied step of the ensemble (one lane per step size)
    if (tid < 64) {
        const unsigned long long occ = __ballot(cnt_b > 0);
        if (tid == 0) s_bm = occ ? __builtin_ctzll(occ) : 64;
    }
    __syncthreads();
    const int bm = s_bm;
    int64_t Tn = INT64_MAX;
    int zn = -1;
    if (bm < 64) {
        Tn = ((Tlast >> bm) + 1) << bm;
        if (Tn <= L.T_end) zn = __builtin_ctzll((unsigned long long)Tn);
    }
    // thread t owns clusters [c0, c1): their counts, then their first positions
    const int per = (C + kWG - 1) / kWG;
    const int c0 = tid * per < C ? tid * per : C;
    const int c1 = c0 + per < C ? c0 + per : C;
    int32_t loc = 0;
    for (int c = c0; c < c1; ++c) {
        const int32_t k = zn >= 0 ? L.ccum[c * 64 + zn] : 0;
        s_start[c] = k;
        loc += k;
    }
    int32_t na;
    int32_t run = block_exscan_i32(loc, s_scan, &na);
    for (int c = c0; c < c1; ++c) {
        const int32_t k = s_start[c];
        s_start[c] = run;
        run += k;
    }
    if (tid == 0) s_start[C] = na;
    __syncthreads();
    for (int c = g; c < C; c += G) {
        const int32_t st = s_start[c], cnt = s_start[c + 1] - st;
        const int32_t* src = L.perm + s_off[c];
        for (int32_t k = tid; k < cnt; k += kWG) {
            L.idx[st + k] = (c == g && k < kWG) ? pre : src[k];
            sa.act_cluster[st + k] = c;
        }
        if (tid == 0) {
            L.cna[c] = cnt;
            L.cst[c] = st;
        }
    }
    if (g != 0) return;
    if (tid == 0) {
        *L.T = Tn;
        *L.na = na;
        count_step(L.counters, Tn, na);
    }
    plan_body(sa, na, s_start, s_off);
}

// ---- predictor (equations (xpred), (vpred)) -----------------------------
__global__ void __launch_bounds__(kWG) predict_kernel(int64_t n, const int64_t* __restrict__ t,
                                                      const int64_t* T_dev, int64_t T_host,
                                                      const int32_t* n_act_dev,
                                                      PredictArgs pa)
{
    if (n_act_dev && *n_act_dev == 0) return;
    const int64_t T = T_dev ? *T_dev : T_host;
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    predict_one(n, i, T, t, pa);
}

// ---- timestep: Aarseth criterion and power-of-two quantisation ----------
__device__ __forceinline__ double norm3(double a, double b, double c)
{
    return sqrt(fma(a, a, fma(b, b, c * c)));
}

__device__ int64_t quantize_dt(double crit, int k_old, int64_t T, int tick_bits,
                               int k_min, int k_max, int* clamped)
{
    int k;
    *clamped = 0;
    if (__builtin_isnan(crit) || __builtin_isinf(crit)) {
        k = k_min;
    } else if (crit <= 0.0) {
        k = k_max;
        *clamped = 1;
    } else {
        int e;
        frexp(crit, &e);            // crit in [2^(e-1), 2^e)
        k = 1 - e;
        if (k < k_min) k = k_min;
        if (k > k_max) { k = k_max; *clamped = 1; }
    }
    if (k_old >= 0 && k < k_old - 1) k = k_old - 1;
    while (k < k_max && (T & ((((int64_t)1) << (tick_bits - k)) - 1)) != 0) ++k;
    return ((int64_t)1) << (tick_bits - k);
}

// ---- corrector + next step (procedure steps 5-8) -------------------------
// The pre-step state of an active particle that the corrector reads, loaded
// before the new forces are summed so that these loads overlap the sum's.
struct OldState {
    int i;                      // particle index
    int64_t t, dt;
    double x[3], v[3];          // x, v (prediction in place) or xp, vp
    double a[3], j[3];
};

__device__ __forceinline__ void load_old_i(const CorrectArgs& c, int i, OldState& o)
{
    const int64_t n = c.n;
    o.i = i;
    o.dt = c.dt[i];
    o.t = c.t[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t q = d * n + i;
        o.x[d] = c.predict_i ? c.x[q] : c.xp[q];
        o.v[d] = c.predict_i ? c.v[q] : c.vp[q];
        o.a[d] = c.a[q];
        o.j[d] = c.j[q];
    }
}

__device__ __forceinline__ void load_old(const CorrectArgs& c, int p, OldState& o)
{
    load_old_i(c, c.idx ? c.idx[p] : p, o);
}

// a1, j1: the new acceleration and jerk of active position p, whose
// pre-step state is o.
__device__ void correct_one(const CorrectArgs& c, int p, const OldState& o, int64_t T,
                            const double a1v[3], const double j1v[3], double pot1, bool have_pot)
{
    const int64_t n = c.n;
    const int i = o.i;
    const double tick = ldexp(1.0, -c.tick_bits);
    const int64_t dt_old = o.dt;
    const double h = (double)dt_old * tick;
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    double s1[3], cc[3], xp[3], vp[3];
    if (c.predict_i) {
        // equations (xpred), (vpred) for this particle, dt = T - t_i
        const double hp = (double)(T - o.t) * tick;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double ac = o.a[d], jk = o.j[d];
            xp[d] = fma(hp, fma(hp, fma(hp, jk * (1.0 / 6.0), ac * 0.5), o.v[d]), o.x[d]);
            vp[d] = fma(hp, fma(hp, jk * 0.5, ac), o.v[d]);
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xp[d] = o.x[d];
            vp[d] = o.v[d];
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t q = d * n + i;
        const double a0 = o.a[d], j0 = o.j[d];
        const double a1 = a1v[d], j1 = j1v[d];
        const double da = a0 - a1;
        const double s0 = 2.0 * (-3.0 * da - (2.0 * j0 + j1) * h) / h2;
        const double c0 = 6.0 * (2.0 * da + (j0 + j1) * h) / h3;
        c.x[q] = xp[d] + s0 * h4 / 24.0 + c0 * h5 / 120.0;
        c.v[q] = vp[d] + s0 * h3 / 6.0 + c0 * h4 / 24.0;
        c.a[q] = a1;
        c.j[q] = j1;
        s1[d] = fma(c0, h, s0);
        cc[d] = c0;
    }
    if (have_pot) c.pot[i] = pot1;
    c.t[i] = T;
    const double A = norm3(a1v[0], a1v[1], a1v[2]);
    const double J = norm3(j1v[0], j1v[1], j1v[2]);
    const double S = norm3(s1[0], s1[1], s1[2]);
    const double Cn = norm3(cc[0], cc[1], cc[2]);
    const double R = (A * S + J * J) / (J * Cn + S * S);
    const double crit = c.form == 0 ? c.eta * sqrt(R) : sqrt(c.eta * R);
    if (c.crit_out) c.crit_out[p] = crit;
    const int k_old = c.tick_bits - log2_step(dt_old);
    int cl;
    const int64_t dt_new = quantize_dt(crit, k_old, T, c.tick_bits, c.k_min, c.k_max, &cl);
    c.dt[i] = dt_new;
    if (c.lv_out) c.lv_out[p] = (uint8_t)log2_step(dt_new);
    if (cl && c.counters) atomicAdd((unsigned long long*)&c.counters[2], 1ull);
}

__global__ void __launch_bounds__(kWG) correct_kernel(CorrectArgs c)
{
    const int na = c.n_act_dev ? *c.n_act_dev : c.n_act_max;
    const int p = blockIdx.x * kWG + threadIdx.x;
    if (p >= na) return;
    const int64_t T = c.T_dev ? *c.T_dev : c.T_host;
    const int64_t st = c.n_act_max;
    OldState o;
    load_old(c, p, o);
    double a1[3], j1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a1[d] = c.acc1[d * st + p];
        j1[d] = c.jrk1[d * st + p];
    }
    correct_one(c, p, o, T, a1, j1, c.pot1 ? c.pot1[p] : 0.0, c.pot1 != nullptr);
}

// The block-step corrector: sums the sweep's j-chunk partials of position p
// in fixed order (the reduce stage) and corrects in the same kernel.
// Grid-stride: a thread per particle for few chunks, a wave for many.
// The particle index (and, for ensembles, the cluster) of a thread's or a
// wave's first position, loaded together with the plan: neither depends on
// it, and the first position's state and partial sums then need one round
// trip after the plan instead of two.
struct FirstPos {
    int p, i, cl;   // cl: the cluster from the selection's record, or -1
};

__device__ __forceinline__ FirstPos first_pos(const CorrectArgs& c, const SweepArgs& sa, int p)
{
    const int q = p < c.n_act_max ? p : c.n_act_max - 1;
    FirstPos f;
    f.p = p;
    f.i = c.idx ? c.idx[q] : q;
    f.cl = (sa.n_clusters > 1 && sa.act_cluster) ? sa.act_cluster[q] : -1;
    return f;
}

__device__ __forceinline__ int first_chunks(const SweepArgs& sa, const FirstPos& f, int p)
{
    return (p == f.p && f.cl >= 0) ? sa.chunks[f.cl] : chunks_of(sa, p);
}

__device__ void correct_reduce_body(const CorrectArgs& c, const SweepArgs& sa, int na,
                                    FirstPos ft, FirstPos fw)
{
    if (c.na_seen && blockIdx.x == 0 && threadIdx.x == 0) *c.na_seen = na;
    const int64_t T = c.T_dev ? *c.T_dev : c.T_host;
    if (thread_reduce(sa.plan->s_max, na)) {
        for (int p = ft.p; p < na; p += gridDim.x * kWG) {
            OldState o;
            load_old_i(c, p == ft.p ? ft.i : (c.idx ? c.idx[p] : p), o);
            double s[kRows];
            reduce_partials_ch(sa, na, p, first_chunks(sa, ft, p), s);
            const double a1[3] = {s[0], s[1], s[2]};
            const double j1[3] = {s[3], s[4], s[5]};
            correct_one(c, p, o, T, a1, j1, s[6], true);
        }
    } else {
        const int lane = threadIdx.x & 63;
        const int wpb = kWG / 64;
        for (int p = fw.p; p < na; p += gridDim.x * wpb) {
            OldState o;
            // the same address in every lane of the wave
            load_old_i(c, p == fw.p ? fw.i : (c.idx ? c.idx[p] : p), o);
            double s[kRows];
            reduce_partials_wave_ch(sa, na, p, first_chunks(sa, fw, p), lane, s);
            if (lane == 0) {
                const double a1[3] = {s[0], s[1], s[2]};
                const double j1[3] = {s[3], s[4], s[5]};
                correct_one(c, p, o, T, a1, j1, s[6], true);
            }
        }
    }
}

__device__ __forceinline__ void correct_reduce_entry(const CorrectArgs& c, const SweepArgs& sa)
{
    const FirstPos ft = first_pos(c, sa, blockIdx.x * kWG + (int)threadIdx.x);
    const FirstPos fw = first_pos(c, sa, blockIdx.x * (kWG / 64) + (int)(threadIdx.x >> 6));
    correct_reduce_body(c, sa, sa.plan->n_act, ft, fw);
}

__global__ void __launch_bounds__(kWG) correct_reduce_kernel(CorrectArgs c, SweepArgs sa)
{
    correct_reduce_entry(c, sa);
}

// The block-step corrector of a refined mixed sweep: the mixed sums from
// the compact outputs, or, for a flagged position, the FP64 refine
// sweep's partials summed in chunk order.  A block the plan put in FP64
// (fp64_all: the refine sweep swept all of it, in list order) is reduced
// from the refine sweep's partials, as correct_reduce_kernel does.
__global__ void __launch_bounds__(kWG) correct_refine_kernel(CorrectArgs c, SweepArgs a,
                                                             SweepArgs ra)
{
    if (a.plan->fp64_all) {
        correct_reduce_entry(c, ra);
        return;
    }
    const int na = *c.n_act_dev;
    if (c.na_seen && blockIdx.x == 0 && threadIdx.x == 0) *c.na_seen = na;
    const int64_t T = c.T_dev ? *c.T_dev : c.T_host;
    const int64_t st = c.n_act_max;
    const int cnt = ra.plan->n_act;
    const int lane = threadIdx.x & 63;
    // rounds of whole waves: a flagged lane's refine chunks are summed by
    // its wave together
    for (int base = (blockIdx.x * kWG + (int)threadIdx.x) & ~63; base < na;
         base += gridDim.x * kWG) {
        const int p = base + lane;
        const int k = p < na ? ra.ref_pos[p] : -1;
        double a1[3], j1[3], pot1 = 0.0;
        OldState o;
        if (p < na) {
            load_old(c, p, o);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a1[d] = c.acc1[d * st + p];
                j1[d] = c.jrk1[d * st + p];
            }
            pot1 = c.pot1[p];
        }
        uint64_t fl = __ballot(k >= 0);
        while (fl) {
            const int owner = __builtin_ctzll(fl);
            fl &= fl - 1;
            const int kf = __shfl(k, owner);
            double s[kRows];
            reduce_partials_wave(ra, cnt, kf, lane, s);
            if (lane == owner) {
                a1[0] = s[0]; a1[1] = s[1]; a1[2] = s[2];
                j1[0] = s[3]; j1[1] = s[4]; j1[2] = s[5];
                pot1 = s[6];
            }
        }
        if (p < na) correct_one(c, p, o, T, a1, j1, pot1, true);
    }
}

__global__ void __launch_bounds__(kWG) init_dt_kernel(int64_t n, int tick_bits,
                                                      const double* a, const double* j,
                                                      int64_t* t, int64_t* dt,
                                                      double eta_s, int k_min,
                                                      int k_max, int64_t* counters)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    const double A = norm3(a[i], a[n + i], a[2 * n + i]);
    const double J = norm3(j[i], j[n + i], j[2 * n + i]);
    const double crit = eta_s * A / J;
    int cl;
    t[i] = 0;
    dt[i] = quantize_dt(crit, -1, 0, tick_bits, k_min, k_max, &cl);
    if (cl && counters) atomicAdd((unsigned long long*)&counters[2], 1ull);
}

__global__ void __launch_bounds__(kWG) copy2_kernel(int64_t count, const double* s0,
                                                    double* d0, const double* s1,
                                                    double* d1)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= count) return;
    d0[i] = s0[i];
    d1[i] = s1[i];
}

// ---- energy: K = 1/2 sum m v^2, W = 1/2 sum m phi, per cluster -----------
__global__ void __launch_bounds__(kWG) energy_reduce_kernel(int64_t n,
                                                            const int64_t* offsets,
                                                            const double* m,
                                                            const double* v,
                                                            const double* phi,
                                                            double* out)
{
    __shared__ double sk[kWG], sw[kWG];
    const int c = blockIdx.x;
    const int64_t b = offsets ? offsets[c] : 0;
    const int64_t e = offsets ? offsets[c + 1] : n;
    double K = 0.0, W = 0.0;
    for (int64_t i = b + threadIdx.x; i < e; i += kWG) {
        const double v2 = fma(v[i], v[i], fma(v[n + i], v[n + i], v[2 * n + i] * v[2 * n + i]));
        K = fma(0.5 * m[i], v2, K);
        W = fma(0.5 * m[i], phi[i], W);
    }
    sk[threadIdx.x] = K;
    sw[threadIdx.x] = W;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sk[threadIdx.x] += sk[threadIdx.x + s];
            sw[threadIdx.x] += sw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * c] = sk[0];
        out[2 * c + 1] = sw[0];
    }
}

__global__ void __launch_bounds__(kWG) iota_kernel(int32_t count, int32_t* out)
{
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i < count) out[i] = i;
}

inline int nblocks(int64_t count, int per)
{
    return (int)((count + per - 1) / per);
}

}  // namespace

int select_blocks(int64_t n) { return nblocks(n, kSelBlock); }

hipError_t launch_select(int64_t n, const int64_t* t, const int64_t* dt,
                         int64_t T_end, int32_t* idx, int32_t* n_act,
                         int64_t* T, int64_t* block_min, int32_t* block_cnt,
                         int64_t* counters, hipStream_t st)
{
    const int nb = nblocks(n, kSelBlock);
    hipLaunchKernelGGL(sel_min_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt, block_min);
    hipLaunchKernelGGL(sel_count_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                       (const int64_t*)block_min, nb, block_cnt, T);
    hipLaunchKernelGGL(sel_write_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                       (const int32_t*)block_cnt, nb, (const int64_t*)T, T_end, idx,
                       n_act, counters);
    return hipGetLastError();
}

hipError_t launch_predict(int64_t n, int tick_bits, const double* x,
                          const double* v, const double* a, const double* j,
                          const int64_t* t, const int64_t* T_dev,
                          int64_t T_host, const int32_t* n_act_dev,
                          double* xp, double* vp, hipStream_t st)
{
    PredictArgs pa{ldexp(1.0, -tick_bits), x, v, a, j, xp, vp};
    hipLaunchKernelGGL(predict_kernel, dim3(nblocks(n, kWG)), dim3(kWG), 0, st, n, t, T_dev,
                       T_host, n_act_dev, pa);
    return hipGetLastError();
}

hipError_t launch_step_select(int64_t n, const int64_t* t, const int64_t* dt, int64_t T_end,
                              int32_t* idx, int32_t* n_act, int64_t* T, int64_t* block_min,
                              int32_t* block_cnt, int64_t* counters, uint32_t* ticket,
                              const SweepArgs& sa, hipStream_t st)
{
    const int nb = nblocks(n, kSelBlock);
    if (nb == 1) {
        hipLaunchKernelGGL(sel_single_plan_kernel, dim3(1), dim3(kWG), 0, st, n, t, dt, T_end,
                           idx, n_act, T, counters, sa);
        return hipGetLastError();
    }
    if (nb <= kSelTicketMax) {
        hipLaunchKernelGGL(sel_min_count_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                           block_min, block_cnt, nb, T, ticket + 1);
        hipLaunchKernelGGL(sel_write_plan_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                           (const int32_t*)block_cnt, nb, (const int64_t*)T, T_end, idx, n_act,
                           counters, sa, ticket);
    } else {
        // many blocks: the standalone selection's passes (no tickets), the
        // list with the clusters' runs, then the plan
        hipLaunchKernelGGL(sel_min_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt, block_min);
        hipLaunchKernelGGL(sel_count_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                           (const int64_t*)block_min, nb, block_cnt, T);
        hipLaunchKernelGGL(sel_write_list_kernel, dim3(nb), dim3(kWG), 0, st, n, t, dt,
                           (const int32_t*)block_cnt, nb, (const int64_t*)T, T_end, idx, n_act,
                           counters, sa);
        hipLaunchKernelGGL(sel_plan_kernel, dim3(1), dim3(kWG), 0, st, sa,
                           (const int32_t*)n_act);
    }
    return hipGetLastError();
}

static int level_grid(int64_t n)
{
    const int g = nblocks(n, kWG * 8);
    return g < 1 ? 1 : (g > 2048 ? 2048 : g);
}

hipError_t launch_level_count(const LevelArgs& L, hipStream_t st)
{
    hipLaunchKernelGGL(level_count_kernel, dim3(level_grid(L.n)), dim3(kWG), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_level_build(const LevelArgs& L, hipStream_t st)
{
    if (L.n_clusters > 1)
        hipLaunchKernelGGL(cl_build_kernel, dim3(L.n_clusters), dim3(kWG), 0, st, L);
    else
        hipLaunchKernelGGL(level_build_kernel, dim3(level_grid(L.n)), dim3(kWG), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_level_select(const LevelArgs& L, const SweepArgs& sa, hipStream_t st)
{
    if (L.n_clusters > 1) {
        hipLaunchKernelGGL(cl_resort_kernel, dim3(L.n_clusters), dim3(kWG), 0, st, L);
        const int grid = L.n_clusters < kSelectGrid ? L.n_clusters : kSelectGrid;
        hipLaunchKernelGGL(cl_select_kernel, dim3(grid), dim3(kWG), 0, st, L, sa);
    } else {
        hipLaunchKernelGGL(level_select_kernel, dim3(1), dim3(kWG), 0, st, L, sa);
    }
    return hipGetLastError();
}

hipError_t launch_correct_reduce(const CorrectArgs& c, const SweepArgs& sa, hipStream_t st)
{
    hipLaunchKernelGGL(correct_reduce_kernel, dim3(reduce_grid(c.n_act_max)), dim3(kWG), 0,
                       st, c, sa);
    return hipGetLastError();
}

hipError_t launch_correct_refine(const CorrectArgs& c, const SweepArgs& a, const SweepArgs& ra,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(correct_refine_kernel, dim3(reduce_grid(c.n_act_max)), dim3(kWG), 0, st,
                       c, a, ra);
    return hipGetLastError();
}

hipError_t launch_correct(const CorrectArgs& c, hipStream_t st)
{
    hipLaunchKernelGGL(correct_kernel, dim3(nblocks(c.n_act_max, kWG)), dim3(kWG), 0,
                       st, c);
    return hipGetLastError();
}

hipError_t launch_init_dt(int64_t n, int tick_bits, const double* a,
                          const double* j, int64_t* t, int64_t* dt,
                          double eta, int form, double eta_init, int k_min, int k_max,
                          int64_t* counters, hipStream_t st)
{
    // start-up factor: the steady one unless the caller gives a smaller one
    // (|a|/|j| has no guard against a small initial jerk)
    const double eta_f = form == 0 ? eta : sqrt(eta);
    const double eta_s = eta_init > 0.0 ? eta_init : eta_f;
    hipLaunchKernelGGL(init_dt_kernel, dim3(nblocks(n, kWG)), dim3(kWG), 0, st, n,
                       tick_bits, a, j, t, dt, eta_s, k_min, k_max, counters);
    return hipGetLastError();
}

hipError_t launch_copy2(int64_t count, const double* src0, double* dst0,
                        const double* src1, double* dst1, hipStream_t st)
{
    hipLaunchKernelGGL(copy2_kernel, dim3(nblocks(count, kWG)), dim3(kWG), 0, st,
                       count, src0, dst0, src1, dst1);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t count, int32_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(iota_kernel, dim3(nblocks(count, kWG)), dim3(kWG), 0, st, count,
                       out);
    return hipGetLastError();
}

// Sets *flag when any of the 12 n values of x, v, a, j is not finite
// (grid-stride; one non-returning atomic per wave that saw one).
__global__ void __launch_bounds__(kWG) nonfinite_kernel(int64_t count, const double* x,
                                                        const double* v, const double* a,
                                                        const double* j, int32_t* flag)
{
    bool bad = false;
    for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * kWG) {
        bad |= !__builtin_isfinite(x[k]) || !__builtin_isfinite(v[k]) ||
               !__builtin_isfinite(a[k]) || !__builtin_isfinite(j[k]);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_finite(int64_t n, const double* x, const double* v, const double* a,
                               const double* j, int32_t* flag, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    const int64_t count = 3 * n;
    const int64_t nb = nblocks(count, kWG);
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(kWG), 0,
                       st, count, x, v, a, j, flag);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(int64_t n, int n_clusters,
                                const int64_t* offsets, const double* m,
                                const double* v, const double* phi,
                                double* out, hipStream_t st)
{
    hipLaunchKernelGGL(energy_reduce_kernel, dim3(n_clusters), dim3(kWG), 0, st, n,
                       offsets, m, v, phi, out);
    return hipGetLastError();
}

}  // namespace hm
