// The O(N_act * N) force / jerk / potential sweep on gfx950 (CDNA4).
//
// Equations (acc), (jrk), (pot) of Section 2: for every active i,
//   a_i   = sum_{j != i} m_j r / s^{3/2}
//   jrk_i = sum_{j != i} m_j / s^{3/2} (v - 3 (r.v) / s  r)
//   phi_i = -sum_{j != i} m_j / s^{1/2}
// with r = x_j - x_i, v = v_j - v_i, s = r^2 + eps^2.
//
// Design (GPU analogue of the paper's i-in-registers, j-streamed loop of
// Section 3.3):
//  * Work is a list of items (cluster, i-tile, j-chunk) that the plan builds
//    on the device.  A persistent grid takes them round-robin (workgroup w
//    takes w, w + grid, ...), so one launch serves any active count, ragged
//    clusters and graph replays.
//  * Each lane holds one or two active particles in registers.  When the active
//    block is small, L lanes of a wave share one particle and take every
//    L-th j; their sums are combined by a wave-shuffle butterfly.  Larger
//    splits go across workgroups (j-chunks) and are added in a fixed order
//    by the reduce kernel, so results are bitwise reproducible.
//  * j-particles stream through LDS in tiles of kTJ, loaded with coalesced
//    SoA reads; all lanes of a wave read the same LDS word when L = 1.
//  * Self-interaction is removed by comparing indices (Section 3.3, the
//    MASK block), but only in tiles that contain one of the wave's i.
//  * Sums are blocked: a tile (FP64) or a run of K j (mixed) is summed
//    into fresh accumulators before it is added to the running sum, which
//    keeps rounding growth near sqrt(N/K) + sqrt(K) instead of sqrt(N).
//
// Precisions:
//  FP64     all arithmetic binary64; 1/sqrt(s) from v_rsq_f64 refined by
//           one third-order Newton step (Section 3.2's iteration taken one
//           order further), ~1 ulp.
//  MIXED    r and v subtracted in FP64 and rounded to FP32; s, 1/sqrt(s)
//           (v_rsq_f32), and the pair terms in FP32; K-term FP32 partial
//           sums added to FP64 running sums.
//  MIXED_2F as MIXED, with the running sums held as two FP32 words
//           (hi + lo) updated by Knuth's TwoSum.
//  MIXED_SP the precision split of Section 3.2 as printed: r subtracted in
//           FP64, velocities rounded to FP32 and subtracted in FP32, the
//           acceleration and potential summed as in MIXED, the jerk kept in
//           one FP32 running sum per lane for the whole j-range.
#include "hermite_internal.h"
#include "plan.h"

#include <type_traits>

namespace hm {
namespace {

constexpr int kMixedK = 16;   // FP32 run length before an FP64 flush

__device__ __forceinline__ double rsqrt_f64(double s)
{
    // y0 from the hardware; with e = 1 - s y0^2,
    // 1/sqrt(s) = y0 (1 - e)^{-1/2} = y0 (1 + e/2 + 3 e^2 / 8 + ...).
    const double y = __builtin_amdgcn_rsq(s);
    const double h = s * y;
    const double e = fma(-h, y, 1.0);
    const double p = fma(e, 0.375, 0.5);
    return fma(y * e, p, y);
}

__global__ void __launch_bounds__(kWG) plan_kernel(SweepArgs a)
{
    plan_body(a, a.n_act_dev ? *a.n_act_dev : a.n_act_max);
}

// ------------------------------------------------------------------------
// Accumulators and pair interactions
// ------------------------------------------------------------------------
struct I64 {   // i-particle in FP64
    double x, y, z, vx, vy, vz;
};

struct SumD {  // FP64 sums: acc, jerk, sum of m/r
    double ax, ay, az, jx, jy, jz, pp;
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = pp = 0.0;
    }
    __device__ __forceinline__ void add(const SumD& o)
    {
        ax += o.ax; ay += o.ay; az += o.az;
        jx += o.jx; jy += o.jy; jz += o.jz;
        pp += o.pp;
    }
};

struct SumF {  // FP32 run sums
    float ax, ay, az, jx, jy, jz, pp;
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = pp = 0.0f;
    }
};

struct TwoF {  // one two-float running sum
    float hi, lo;
    __device__ __forceinline__ void add(float b)
    {
        const float s = hi + b;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (b - bb);
        hi = s;
        lo += err;
    }
    __device__ __forceinline__ double value() const
    {
        return (double)hi + (double)lo;
    }
};

struct Sum2F {
    TwoF ax, ay, az, jx, jy, jz, pp;
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = pp = TwoF{0.0f, 0.0f};
    }
};

// One FP64 pair term: with b3 = 3 (r.v) / s,
//   acc += m/s^{3/2} r,  jerk += m/s^{3/2} (v - b3 r),  pp += m/s^{1/2}.
template <bool MASK>
__device__ __forceinline__ void pair_f64(const I64& I, double eps2, double xj,
                                         double yj, double zj, double vxj,
                                         double vyj, double vzj, double mj,
                                         bool self, SumD& S)
{
    const double dx = xj - I.x, dy = yj - I.y, dz = zj - I.z;
    const double dvx = vxj - I.vx, dvy = vyj - I.vy, dvz = vzj - I.vz;
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
    double ri = rsqrt_f64(r2);
    if (MASK) ri = self ? 0.0 : ri;
    const double mr = mj * ri;
    const double ri2 = ri * ri;
    const double mr3 = mr * ri2;
    const double rv = fma(dx, dvx, fma(dy, dvy, dz * dvz));
    const double b3 = (rv * ri2) * 3.0;
    S.pp += mr;
    S.ax = fma(mr3, dx, S.ax);
    S.ay = fma(mr3, dy, S.ay);
    S.az = fma(mr3, dz, S.az);
    S.jx = fma(mr3, fma(-b3, dx, dvx), S.jx);
    S.jy = fma(mr3, fma(-b3, dy, dvy), S.jy);
    S.jz = fma(mr3, fma(-b3, dz, dvz), S.jz);
}

template <bool MASK>
__device__ __forceinline__ void pot_f64(const I64& I, double eps2, double xj,
                                        double yj, double zj, double mj,
                                        bool self, SumD& S)
{
    const double dx = xj - I.x, dy = yj - I.y, dz = zj - I.z;
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
    double ri = rsqrt_f64(r2);
    if (MASK) ri = self ? 0.0 : ri;
    S.pp = fma(mj, ri, S.pp);
}

// One mixed-precision pair term: FP64 differences, FP32 pair arithmetic.
template <bool MASK>
__device__ __forceinline__ void pair_mixed(const I64& I, float eps2f, double xj,
                                           double yj, double zj, double vxj,
                                           double vyj, double vzj, float mj,
                                           bool self, SumF& S)
{
    const float dx = (float)(xj - I.x), dy = (float)(yj - I.y), dz = (float)(zj - I.z);
    const float dvx = (float)(vxj - I.vx), dvy = (float)(vyj - I.vy),
                dvz = (float)(vzj - I.vz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
    float ri = __builtin_amdgcn_rsqf(r2);
    if (MASK) ri = self ? 0.0f : ri;
    const float mr = mj * ri;
    const float ri2 = ri * ri;
    const float mr3 = mr * ri2;
    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float b3 = (rv * ri2) * 3.0f;
    S.pp += mr;
    S.ax = fmaf(mr3, dx, S.ax);
    S.ay = fmaf(mr3, dy, S.ay);
    S.az = fmaf(mr3, dz, S.az);
    S.jx = fmaf(mr3, fmaf(-b3, dx, dvx), S.jx);
    S.jy = fmaf(mr3, fmaf(-b3, dy, dvy), S.jy);
    S.jz = fmaf(mr3, fmaf(-b3, dz, dvz), S.jz);
}

// Split form of the mixed pair term: every FP64 coordinate c is held as
// hi = fl32(c), lo = fl32(c - hi), and the difference is formed in FP32 as
// (hi_j - hi_i) + (lo_j - lo_i).  For a close pair the hi difference is
// exact (Sterbenz), so the result carries the same FP32 rounding of the
// FP64 difference as the cast form, at three FP32 operations instead of
// an FP64 subtraction and a conversion.
struct I32S {  // i-particle, split coordinates
    float xh, xl, yh, yl, zh, zl, vxh, vxl, vyh, vyl, vzh, vzl;
};

__device__ __forceinline__ void split(double c, float& h, float& l)
{
    h = (float)c;
    l = (float)(c - (double)h);
}

template <bool MASK>
__device__ __forceinline__ void pair_split(const I32S& I, float eps2f, const float* J,
                                           float mj, bool self, SumF& S)
{
    const float dx = (J[0] - I.xh) + (J[1] - I.xl);
    const float dy = (J[2] - I.yh) + (J[3] - I.yl);
    const float dz = (J[4] - I.zh) + (J[5] - I.zl);
    const float dvx = (J[6] - I.vxh) + (J[7] - I.vxl);
    const float dvy = (J[8] - I.vyh) + (J[9] - I.vyl);
    const float dvz = (J[10] - I.vzh) + (J[11] - I.vzl);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
    float ri = __builtin_amdgcn_rsqf(r2);
    if (MASK) ri = self ? 0.0f : ri;
    const float mr = mj * ri;
    const float ri2 = ri * ri;
    const float mr3 = mr * ri2;
    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float b3 = (rv * ri2) * 3.0f;
    S.pp += mr;
    S.ax = fmaf(mr3, dx, S.ax);
    S.ay = fmaf(mr3, dy, S.ay);
    S.az = fmaf(mr3, dz, S.az);
    S.jx = fmaf(mr3, fmaf(-b3, dx, dvx), S.jx);
    S.jy = fmaf(mr3, fmaf(-b3, dy, dvy), S.jy);
    S.jz = fmaf(mr3, fmaf(-b3, dz, dvz), S.jz);
}

// Paper-faithful mixed term (Section 3.2 as printed): velocities held in
// FP32 and their difference taken in FP32; everything else as pair_mixed.
struct I64SP {  // i-particle: FP64 position, FP32 velocity
    double x, y, z;
    float vx, vy, vz;
};

template <bool MASK>
__device__ __forceinline__ void pair_sp(const I64SP& I, float eps2f, double xj, double yj,
                                        double zj, float vxj, float vyj, float vzj, float mj,
                                        bool self, SumF& S)
{
    const float dx = (float)(xj - I.x), dy = (float)(yj - I.y), dz = (float)(zj - I.z);
    const float dvx = vxj - I.vx, dvy = vyj - I.vy, dvz = vzj - I.vz;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
    float ri = __builtin_amdgcn_rsqf(r2);
    if (MASK) ri = self ? 0.0f : ri;
    const float mr = mj * ri;
    const float ri2 = ri * ri;
    const float mr3 = mr * ri2;
    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float b3 = (rv * ri2) * 3.0f;
    S.pp += mr;
    S.ax = fmaf(mr3, dx, S.ax);
    S.ay = fmaf(mr3, dy, S.ay);
    S.az = fmaf(mr3, dz, S.az);
    S.jx = fmaf(mr3, fmaf(-b3, dx, dvx), S.jx);
    S.jy = fmaf(mr3, fmaf(-b3, dy, dvy), S.jy);
    S.jz = fmaf(mr3, fmaf(-b3, dz, dvz), S.jz);
}

// Flush of the paper-faithful mode: acceleration and potential runs go to
// the FP64 sums, the jerk stays in its FP32 accumulator (never flushed).
__device__ __forceinline__ void flush_keep_jerk(SumF& f, SumD& d)
{
    d.ax += (double)f.ax; d.ay += (double)f.ay; d.az += (double)f.az;
    d.pp += (double)f.pp;
    f.ax = f.ay = f.az = f.pp = 0.0f;
}

__device__ __forceinline__ void flush(SumF& f, SumD& d)
{
    d.ax += (double)f.ax; d.ay += (double)f.ay; d.az += (double)f.az;
    d.jx += (double)f.jx; d.jy += (double)f.jy; d.jz += (double)f.jz;
    d.pp += (double)f.pp;
    f.zero();
}

__device__ __forceinline__ void flush(SumF& f, Sum2F& d)
{
    d.ax.add(f.ax); d.ay.add(f.ay); d.az.add(f.az);
    d.jx.add(f.jx); d.jy.add(f.jy); d.jz.add(f.jz);
    d.pp.add(f.pp);
    f.zero();
}

// LDS tile of j-particles (SoA).  Masses are FP32 in the mixed paths.
template <typename MT>
struct Tile {
    double x[kTJ], y[kTJ], z[kTJ], vx[kTJ], vy[kTJ], vz[kTJ];
    MT m[kTJ];
};

// LDS tile of j-particles with split coordinates: c[k][j] for the twelve
// hi/lo words (x, y, z, vx, vy, vz), and the FP32 mass.
struct TileS {
    float c[12][kTJ];
    float m[kTJ];
};

// LDS tile for the paper-faithful mode: FP64 positions, FP32 velocities.
struct TileSP {
    double x[kTJ], y[kTJ], z[kTJ];
    float vx[kTJ], vy[kTJ], vz[kTJ], m[kTJ];
};

// ---- tile loops ---------------------------------------------------------
// Each lane carries IPL active particles; every j read from LDS is used by
// all of them (independent dependency chains, and IPL times fewer LDS
// reads per interaction).
template <bool MASK, int IPL>
__device__ __forceinline__ void tile_f64(const Tile<double>& T, int cnt, int sub,
                                         int L, int64_t tb, const int (&ii)[IPL],
                                         const I64 (&I)[IPL], double eps2, SumD (&S)[IPL])
{
    constexpr int kUnroll = IPL == 1 ? 4 : 2;
    SumD t[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) t[q].zero();
#pragma unroll kUnroll
    for (int jj = sub; jj < cnt; jj += L) {
        const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
        const double vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj], mj = T.m[jj];
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const bool self = MASK && (tb + jj == (int64_t)ii[q]);
            pair_f64<MASK>(I[q], eps2, xj, yj, zj, vxj, vyj, vzj, mj, self, t[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < IPL; ++q) S[q].add(t[q]);
}

template <bool MASK>
__device__ __forceinline__ void tile_pot(const Tile<double>& T, int cnt, int sub,
                                         int L, int64_t tb, int i, const I64& I,
                                         double eps2, SumD& S)
{
    SumD t;
    t.pp = 0.0;
#pragma unroll 4
    for (int jj = sub; jj < cnt; jj += L) {
        const bool self = MASK && (tb + jj == (int64_t)i);
        pot_f64<MASK>(I, eps2, T.x[jj], T.y[jj], T.z[jj], T.m[jj], self, t);
    }
    S.pp += t.pp;
}

template <bool MASK, int IPL, typename RUN>
__device__ __forceinline__ void tile_mixed(const Tile<float>& T, int cnt, int sub,
                                           int L, int64_t tb, const int (&ii)[IPL],
                                           const I64 (&I)[IPL], float eps2f,
                                           SumF (&f)[IPL], RUN (&S)[IPL])
{
    constexpr int kUnroll = IPL == 1 ? 4 : 2;
    const int step = kMixedK * L;
    for (int jb = 0; jb < cnt; jb += step) {
        const int je = (jb + step < cnt) ? jb + step : cnt;
#pragma unroll kUnroll
        for (int jj = jb + sub; jj < je; jj += L) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const double vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj];
            const float mj = T.m[jj];
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                const bool self = MASK && (tb + jj == (int64_t)ii[q]);
                pair_mixed<MASK>(I[q], eps2f, xj, yj, zj, vxj, vyj, vzj, mj, self, f[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < IPL; ++q) flush(f[q], S[q]);
    }
}

template <bool MASK, int IPL, typename RUN>
__device__ __forceinline__ void tile_split(const TileS& T, int cnt, int sub, int L,
                                           int64_t tb, const int (&ii)[IPL],
                                           const I32S (&I)[IPL], float eps2f,
                                           SumF (&f)[IPL], RUN (&S)[IPL])
{
    constexpr int kUnroll = IPL == 1 ? 4 : 2;
    const int step = kMixedK * L;
    for (int jb = 0; jb < cnt; jb += step) {
        const int je = (jb + step < cnt) ? jb + step : cnt;
#pragma unroll kUnroll
        for (int jj = jb + sub; jj < je; jj += L) {
            float J[12];
#pragma unroll
            for (int w = 0; w < 12; ++w) J[w] = T.c[w][jj];
            const float mj = T.m[jj];
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                const bool self = MASK && (tb + jj == (int64_t)ii[q]);
                pair_split<MASK>(I[q], eps2f, J, mj, self, f[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < IPL; ++q) flush(f[q], S[q]);
    }
}

template <bool MASK, int IPL>
__device__ __forceinline__ void tile_sp(const TileSP& T, int cnt, int sub, int L, int64_t tb,
                                        const int (&ii)[IPL], const I64SP (&I)[IPL],
                                        float eps2f, SumF (&f)[IPL], SumD (&S)[IPL])
{
    constexpr int kUnroll = IPL == 1 ? 4 : 2;
    const int step = kMixedK * L;
    for (int jb = 0; jb < cnt; jb += step) {
        const int je = (jb + step < cnt) ? jb + step : cnt;
#pragma unroll kUnroll
        for (int jj = jb + sub; jj < je; jj += L) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const float vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj], mj = T.m[jj];
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                const bool self = MASK && (tb + jj == (int64_t)ii[q]);
                pair_sp<MASK>(I[q], eps2f, xj, yj, zj, vxj, vyj, vzj, mj, self, f[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < IPL; ++q) flush_keep_jerk(f[q], S[q]);
    }
}

__device__ __forceinline__ double shfl_sum(double v, int L)
{
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Final per-lane values: acc xyz, jerk xyz, pot (-sum m/r).
__device__ __forceinline__ void finalize(const SumD& S, double out[7])
{
    out[0] = S.ax; out[1] = S.ay; out[2] = S.az;
    out[3] = S.jx; out[4] = S.jy; out[5] = S.jz;
    out[6] = -S.pp;
}

__device__ __forceinline__ void finalize(const Sum2F& S, double out[7])
{
    out[0] = S.ax.value(); out[1] = S.ay.value(); out[2] = S.az.value();
    out[3] = S.jx.value(); out[4] = S.jy.value(); out[5] = S.jz.value();
    out[6] = -S.pp.value();
}


// ------------------------------------------------------------------------
// The persistent sweep kernel.
//   PREC 0 = FP64, 1 = mixed (FP64 running sums), 2 = mixed two-float.
//   POT_ONLY: potential only, FP64 (energy diagnostic).
//   IPL: active particles per lane (1 or 2).  Lane `slot` of an item holds
//   the item's particles slot, slot + kWG/L, ...
// ------------------------------------------------------------------------
// SEL: the workgroup first selects the block itself (one system of
// n <= kFusedSelMax; the active list stays in LDS) and computes the plan;
// workgroup 0 publishes list, n_act, T, plan and counters for the corrector.
template <int PREC, bool POT_ONLY, int IPL, bool SPLIT, bool SEL = false>
__global__ void __launch_bounds__(kWG) sweep_kernel(SweepArgs a)
{
    static_assert(!SEL || !POT_ONLY, "the fused selection is for block steps");
    static_assert(!SPLIT || (PREC == 1 || PREC == 2), "split form is for the mixed modes");
    using MT = typename std::conditional<PREC == 0, double, float>::type;
    using RUN = typename std::conditional<PREC == 2, Sum2F, SumD>::type;
    using TT = typename std::conditional<
        SPLIT, TileS, typename std::conditional<PREC == 3, TileSP, Tile<MT>>::type>::type;
    __shared__ TT T;
    __shared__ int32_t s_ioff[kLdsClusters + 1];

    // item offsets of the clusters in LDS when they fit (the item -> cluster
    // search then costs no global round trips)
    const bool ioff_lds = a.n_clusters > 1 && a.n_clusters <= kLdsClusters;
    if (ioff_lds) {
        for (int k = threadIdx.x; k <= a.n_clusters; k += kWG) s_ioff[k] = a.item_off[k];
        __syncthreads();
    }

    SweepPlan* P = a.plan;
    const int tid = threadIdx.x;
    int na, L, ti, s_max, total;
    int64_t jc, Tpred;
    const int32_t* idx_lds = nullptr;
    if constexpr (SEL) {
        __shared__ int32_t s_idx[kFusedSelMax];
        na = select_in_lds(a.pred_t, a.sel_dt, a.n, a.sel_T_end, s_idx, &Tpred);
        int32_t L_, ti_;
        plan_split(a, na, 1, &L_, &ti_, &jc);
        L = L_;
        ti = ti_;
        s_max = na > 0 ? (int)((a.n + jc - 1) / jc) : 0;
        total = ((na + ti - 1) / ti) * s_max;
        idx_lds = s_idx;
        if (blockIdx.x == 0) {
            for (int p = tid; p < na; p += kWG) a.sel_idx_out[p] = s_idx[p];
            if (tid == 0) {
                *a.sel_na_out = na;
                *a.sel_T_out = Tpred;
                P->n_act = na;
                P->L = L;
                P->ti = ti;
                P->s_max = s_max;
                P->jc = jc;
                P->total_items = total;
                count_step(a.counters, Tpred, na);
                if (a.counters && na > 0)
                    atomicAdd((unsigned long long*)&a.counters[1],
                              (unsigned long long)((int64_t)na * a.n));
            }
        }
    } else {
        na = P->n_act;
        L = P->L;
        ti = P->ti;
        jc = P->jc;
        s_max = P->s_max;
        total = P->total_items;
        Tpred = a.pred_x ? *a.pred_T : 0;
    }
    if (na == 0) return;
    const int rows = kWG / L;          // lanes' slots per particle row
    const int slot = tid / L;
    const int sub = tid & (L - 1);
    const int C = a.n_clusters;
    const int64_t n = a.n;

    // Workgroup w takes items w, w + grid, w + 2 grid, ...
    int item = blockIdx.x;
    for (;; ) {
        if (item >= total) break;

        // one system: the item layout follows from the plan alone
        int c = 0, local = item;
        if (C > 1) {
            if (ioff_lds) {
                c = upper_bound_i32(s_ioff, C + 1, item) - 1;
                local = item - s_ioff[c];
            } else {
                c = upper_bound_i32(a.item_off, C + 1, item) - 1;
                local = item - a.item_off[c];
            }
        }
        const int ch = (C == 1) ? s_max : a.chunks[c];
        const int tile_i = local / ch;
        const int k = local - tile_i * ch;
        const int p0 = ((C == 1) ? 0 : a.act_start[c]) + tile_i * ti;
        const int rem = ((C == 1) ? na : a.act_cnt[c]) - tile_i * ti;
        const int pcnt = rem < ti ? rem : ti;
        const int64_t cb = (C == 1) ? 0 : a.offsets[c];
        const int64_t ce = (C == 1) ? n : a.offsets[c + 1];
        const int64_t j0 = cb + (int64_t)k * jc;
        const int64_t j1 = (j0 + jc < ce) ? j0 + jc : ce;
        const double eps2 = a.eps2_c ? a.eps2_c[c] : a.eps2;
        const float eps2f = (float)eps2;

        bool valid[IPL];
        int pp[IPL], ii[IPL];
        I64 I[IPL];
        I32S IS[IPL];
        I64SP ISP[IPL];
        RUN S[IPL];
        SumF F[IPL];
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const int pos = slot + q * rows;
            valid[q] = pos < pcnt;
            pp[q] = p0 + (valid[q] ? pos : 0);
            if constexpr (SEL) ii[q] = idx_lds[pp[q]];
            else ii[q] = a.idx ? a.idx[pp[q]] : pp[q];
            double r[3], w[3];
            fetch_particle(a, ii[q], Tpred, r, w);
            I[q].x = r[0]; I[q].y = r[1]; I[q].z = r[2];
            I[q].vx = w[0]; I[q].vy = w[1]; I[q].vz = w[2];
            if constexpr (PREC == 3) {
                ISP[q] = I64SP{I[q].x, I[q].y, I[q].z, (float)I[q].vx, (float)I[q].vy,
                               (float)I[q].vz};
            }
            if constexpr (SPLIT) {
                split(I[q].x, IS[q].xh, IS[q].xl);
                split(I[q].y, IS[q].yh, IS[q].yl);
                split(I[q].z, IS[q].zh, IS[q].zl);
                split(I[q].vx, IS[q].vxh, IS[q].vxl);
                split(I[q].vy, IS[q].vyh, IS[q].vyl);
                split(I[q].vz, IS[q].vzh, IS[q].vzl);
            }
            S[q].zero();
            F[q].zero();
        }

        // j streams through LDS in tiles of kTJ: one cooperative load per
        // tile (a lane reading its own j from global memory instead waits a
        // round trip per j, which measured slower whenever L = 64 chunks
        // were long)
        for (int64_t tb = j0; tb < j1; tb += kTJ) {
            const int cnt = (int)((j1 - tb) < kTJ ? (j1 - tb) : kTJ);
            __syncthreads();
            if (tid < cnt) {
                const int64_t jg = tb + tid;
                if constexpr (POT_ONLY) {
                    T.x[tid] = a.xp[jg];
                    T.y[tid] = a.xp[n + jg];
                    T.z[tid] = a.xp[2 * n + jg];
                    T.m[tid] = (MT)a.m[jg];
                } else {
                    double r[3], w[3];
                    fetch_particle(a, jg, Tpred, r, w);
                    if constexpr (SPLIT) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            split(r[d], T.c[2 * d][tid], T.c[2 * d + 1][tid]);
                            split(w[d], T.c[6 + 2 * d][tid], T.c[7 + 2 * d][tid]);
                        }
                        T.m[tid] = (float)a.m[jg];
                    } else {
                        T.x[tid] = r[0];
                        T.y[tid] = r[1];
                        T.z[tid] = r[2];
                        T.vx[tid] = w[0];   // rounded to FP32 in the paper-faithful mode
                        T.vy[tid] = w[1];
                        T.vz[tid] = w[2];
                        T.m[tid] = (MT)a.m[jg];
                    }
                }
            }
            __syncthreads();
            bool mine = false;
#pragma unroll
            for (int q = 0; q < IPL; ++q)
                mine = mine || ((int64_t)ii[q] >= tb && (int64_t)ii[q] < tb + cnt);
            const bool need_mask = __any(mine);
            if constexpr (POT_ONLY) {
                if (need_mask) tile_pot<true>(T, cnt, sub, L, tb, ii[0], I[0], eps2, S[0]);
                else           tile_pot<false>(T, cnt, sub, L, tb, ii[0], I[0], eps2, S[0]);
            } else if constexpr (PREC == 0) {
                if (need_mask) tile_f64<true, IPL>(T, cnt, sub, L, tb, ii, I, eps2, S);
                else           tile_f64<false, IPL>(T, cnt, sub, L, tb, ii, I, eps2, S);
            } else if constexpr (SPLIT) {
                if (need_mask) tile_split<true, IPL>(T, cnt, sub, L, tb, ii, IS, eps2f, F, S);
                else           tile_split<false, IPL>(T, cnt, sub, L, tb, ii, IS, eps2f, F, S);
            } else if constexpr (PREC == 3) {
                if (need_mask) tile_sp<true, IPL>(T, cnt, sub, L, tb, ii, ISP, eps2f, F, S);
                else           tile_sp<false, IPL>(T, cnt, sub, L, tb, ii, ISP, eps2f, F, S);
            } else {
                if (need_mask) tile_mixed<true, IPL>(T, cnt, sub, L, tb, ii, I, eps2f, F, S);
                else           tile_mixed<false, IPL>(T, cnt, sub, L, tb, ii, I, eps2f, F, S);
            }
        }

#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            double out[7];
            finalize(S[q], out);
            if constexpr (PREC == 3) {
                // the jerk was summed in FP32 over the whole j-chunk
                out[3] = (double)F[q].jx;
                out[4] = (double)F[q].jy;
                out[5] = (double)F[q].jz;
            }
            if (L > 1) {
#pragma unroll
                for (int r = 0; r < 7; ++r) out[r] = shfl_sum(out[r], L);
            }
            if (valid[q] && sub == 0) {
                double* dst = a.partial + (int64_t)k * 7 * na + pp[q];
                if (POT_ONLY) {
                    dst[6 * (int64_t)na] = out[6];
                } else {
#pragma unroll
                    for (int r = 0; r < 7; ++r) dst[r * (int64_t)na] = out[r];
                }
            }
        }
        // further items round-robin: a shared counter would serialise every
        // fetch on one address (tens of ns each across the chip)
        item += (int)gridDim.x;
        __syncthreads();   // the next item restages the LDS tile
    }
}

// Adds the j-chunk partial sums of every active particle in chunk order.
// Grid-stride over particles: one thread each when chunks are few, one
// wave each when they are many (the launch shape does not depend on n_act).
template <bool POT_ONLY>
__device__ __forceinline__ void store_reduced(const SweepArgs& a, int p, const double s[7])
{
    const int64_t st = a.n_act_max;
    if (POT_ONLY) {
        a.pot[p] = s[6];
        return;
    }
    a.acc[p] = s[0];
    a.acc[st + p] = s[1];
    a.acc[2 * st + p] = s[2];
    if (a.jerk) {
        a.jerk[p] = s[3];
        a.jerk[st + p] = s[4];
        a.jerk[2 * st + p] = s[5];
    }
    if (a.pot) a.pot[p] = s[6];
}

template <bool POT_ONLY>
__global__ void __launch_bounds__(kWG) reduce_kernel(SweepArgs a)
{
    const int na = a.plan->n_act;
    if (thread_reduce(a.plan->s_max, na)) {
        for (int p = blockIdx.x * kWG + threadIdx.x; p < na; p += gridDim.x * kWG) {
            double s[7];
            reduce_partials(a, na, p, s);
            store_reduced<POT_ONLY>(a, p, s);
        }
    } else {
        const int lane = threadIdx.x & 63;
        const int wpb = kWG / 64;
        for (int p = blockIdx.x * wpb + (int)(threadIdx.x >> 6); p < na; p += gridDim.x * wpb) {
            double s[7];
            reduce_partials_wave(a, na, p, lane, s);
            if (lane == 0) store_reduced<POT_ONLY>(a, p, s);
        }
    }
}

typedef void (*SweepFn)(SweepArgs);

// The fused select + sweep instantiations (block steps of one small system).
SweepFn sweep_sel_fn(int precision, int variant)
{
    const bool two = (variant & 1) != 0;
    const bool spl = (variant & 2) != 0;
    if (precision == 0)
        return two ? sweep_kernel<0, false, 2, false, true> : sweep_kernel<0, false, 1, false, true>;
    if (precision == 3)
        return two ? sweep_kernel<3, false, 2, false, true> : sweep_kernel<3, false, 1, false, true>;
    if (precision == 1) {
        if (spl) return two ? sweep_kernel<1, false, 2, true, true> : sweep_kernel<1, false, 1, true, true>;
        return two ? sweep_kernel<1, false, 2, false, true> : sweep_kernel<1, false, 1, false, true>;
    }
    if (spl) return two ? sweep_kernel<2, false, 2, true, true> : sweep_kernel<2, false, 1, true, true>;
    return two ? sweep_kernel<2, false, 2, false, true> : sweep_kernel<2, false, 1, false, true>;
}

// variant: bit 0 -> two active particles per lane; bit 1 -> split
// differences (MIXED and MIXED_2F only; FP64 and MIXED_SP ignore it).
SweepFn sweep_fn(int precision, int variant, bool pot_only)
{
    if (pot_only) return sweep_kernel<0, true, 1, false>;
    const bool two = (variant & 1) != 0;
    const bool spl = (variant & 2) != 0;
    if (precision == 0)
        return two ? sweep_kernel<0, false, 2, false> : sweep_kernel<0, false, 1, false>;
    if (precision == 1) {
        if (spl) return two ? sweep_kernel<1, false, 2, true> : sweep_kernel<1, false, 1, true>;
        return two ? sweep_kernel<1, false, 2, false> : sweep_kernel<1, false, 1, false>;
    }
    if (precision == 3)
        return two ? sweep_kernel<3, false, 2, false> : sweep_kernel<3, false, 1, false>;
    if (spl) return two ? sweep_kernel<2, false, 2, true> : sweep_kernel<2, false, 1, true>;
    return two ? sweep_kernel<2, false, 2, false> : sweep_kernel<2, false, 1, false>;
}

}  // namespace

int max_plan_items(const SweepArgs& a)
{
    int best = 0;
    const int32_t top = a.n_act_max < (int32_t)a.n ? a.n_act_max : (int32_t)a.n;
    for (int32_t na = 1; na <= top; ++na) {
        int32_t L, ti;
        int64_t jc;
        plan_split(a, na, 1, &L, &ti, &jc);
        const int64_t items = (int64_t)((na + ti - 1) / ti) * ((a.n + jc - 1) / jc);
        if (items > best) best = (int)items;
    }
    return best > 0 ? best : 1;
}

hipError_t launch_select_sweep(const SweepArgs& a_in, int precision, int variant, int grid,
                               hipStream_t st)
{
    SweepArgs a = a_in;
    a.ipl = (variant & 1) ? 2 : 1;
    hipLaunchKernelGGL(sweep_sel_fn(precision, variant), dim3(grid), dim3(kWG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sweep_only(const SweepArgs& a_in, int precision, int variant, int grid,
                             hipStream_t st)
{
    SweepArgs a = a_in;
    a.ipl = (variant & 1) ? 2 : 1;
    hipLaunchKernelGGL(sweep_fn(precision, variant, false), dim3(grid), dim3(kWG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_force(const SweepArgs& a_in, int precision, int variant,
                        int grid, bool pot_only, hipStream_t st)
{
    SweepArgs a = a_in;
    a.ipl = (!pot_only && (variant & 1)) ? 2 : 1;
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kWG), 0, st, a);
    hipLaunchKernelGGL(sweep_fn(precision, variant, pot_only), dim3(grid), dim3(kWG), 0, st, a);
    const int rgrid = reduce_grid(a.n_act_max);
    if (pot_only) {
        hipLaunchKernelGGL(reduce_kernel<true>, dim3(rgrid), dim3(kWG), 0, st, a);
    } else {
        hipLaunchKernelGGL(reduce_kernel<false>, dim3(rgrid), dim3(kWG), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace hm

namespace hm {

// Resident workgroups per compute unit of a sweep kernel (from its register
// and LDS use); the default persistent grid is this times the CU count.
int sweep_occupancy(int precision, int variant, bool pot_only)
{
    int nb = 0;
    const void* f = reinterpret_cast<const void*>(sweep_fn(precision, variant, pot_only));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWG, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 4;
    }
    return nb;
}

}  // namespace hm
