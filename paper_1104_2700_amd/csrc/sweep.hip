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

// FP32 run lengths before an FP64 flush: kMixedK by default, kMixedKLong
// (variant bit 2) halves the flushes' cost for more FP32 rounding per run
constexpr int kMixedK = 16;
constexpr int kMixedKLong = 32;

#ifndef HM_MIXED_NR
#define HM_MIXED_NR 0
#endif

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

struct SumD {  // FP64 sums: acc, jerk, sum of m/r; FP32 error estimates
    double ax, ay, az, jx, jy, jz, pp;
    float ea, ej;  // sums over FP32 runs of |run sum|^2 (acc, jerk)
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = pp = 0.0;
        ea = ej = 0.0f;
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
    // adds an FP64 value as its two FP32 words
    __device__ __forceinline__ void add_d(double d)
    {
        const float h = (float)d;
        add(h);
        lo += (float)(d - (double)h);
    }
    __device__ __forceinline__ double value() const
    {
        return (double)hi + (double)lo;
    }
};

struct Sum2F {
    TwoF ax, ay, az, jx, jy, jz, pp;
    float ea, ej;  // as in SumD
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = pp = TwoF{0.0f, 0.0f};
        ea = ej = 0.0f;
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


// ---- mixed precision: FP32 pair arithmetic with an FP64 near field ------
//
// With FP32 pair arithmetic every pair term carries a relative error of a
// few u32, and a particle's error is their random walk weighted by the
// terms' magnitudes, i.e. dominated by its nearest neighbours, whose terms
// are the largest.  Pairs closer than the near-field radius (r^2 <= near2:
// a few mean interparticle spacings, set per cluster from its size) are
// therefore evaluated in FP64 instead, in a divergent branch that the wave
// takes only for the few j that are near one of its particles.  The self
// pair (r^2 = eps^2 exactly) always takes that branch, where an index
// compare drops it: no separate masked tile loop is needed.

__device__ __forceinline__ float rsq_f32(float s)
{
    float y = __builtin_amdgcn_rsqf(s);
#if HM_MIXED_NR
    // one Newton step, y (1 + e/2) with e = 1 - s y^2 (Section 3.2)
    const float h = s * y;
    const float e = fmaf(-h, y, 1.0f);
    y = fmaf(y * 0.5f, e, y);
#endif
    return y;
}

// FP64 terms of one near pair from FP64 differences: acc xyz, jerk xyz and
// m/r (the self pair gives zeros).
__device__ __forceinline__ void near_terms(double dx, double dy, double dz, double dvx,
                                           double dvy, double dvz, double mj, double eps2,
                                           bool self, double o[7])
{
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
    const double y = rsqrt_f64(r2);
    const double ri = self ? 0.0 : y;
    const double mr = mj * ri;
    const double ri2 = ri * ri;
    const double mr3 = mr * ri2;
    const double rv = fma(dx, dvx, fma(dy, dvy, dz * dvz));
    const double b3 = (rv * ri2) * 3.0;
    o[0] = mr3 * dx;
    o[1] = mr3 * dy;
    o[2] = mr3 * dz;
    o[3] = mr3 * fma(-b3, dx, dvx);
    o[4] = mr3 * fma(-b3, dy, dvy);
    o[5] = mr3 * fma(-b3, dz, dvz);
    o[6] = mr;
}

__device__ __forceinline__ void add_near(SumD& S, const double o[7])
{
    S.ax += o[0]; S.ay += o[1]; S.az += o[2];
    S.jx += o[3]; S.jy += o[4]; S.jz += o[5];
    S.pp += o[6];
}

__device__ __forceinline__ void add_near(Sum2F& S, const double o[7])
{
    S.ax.add_d(o[0]); S.ay.add_d(o[1]); S.az.add_d(o[2]);
    S.jx.add_d(o[3]); S.jy.add_d(o[4]); S.jz.add_d(o[5]);
    S.pp.add_d(o[6]);
}

// The FP32 part of a mixed pair term, shared by every mixed form.  first:
// the run's first term starts the run sums (no zeroing between runs);
// first_j: the same for the jerk (the paper-faithful mode never restarts
// its jerk sum).
__device__ __forceinline__ void far_terms(float dx, float dy, float dz, float dvx, float dvy,
                                          float dvz, float ri, float mj, bool first,
                                          bool first_j, SumF& S)
{
    const float mr = mj * ri;
    const float ri2 = ri * ri;
    const float mr3 = mr * ri2;
    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float b3 = (rv * ri2) * 3.0f;
    const float jx = fmaf(-b3, dx, dvx), jy = fmaf(-b3, dy, dvy), jz = fmaf(-b3, dz, dvz);
    if (first) {
        S.pp = mr;
        S.ax = mr3 * dx;
        S.ay = mr3 * dy;
        S.az = mr3 * dz;
    } else {
        S.pp += mr;
        S.ax = fmaf(mr3, dx, S.ax);
        S.ay = fmaf(mr3, dy, S.ay);
        S.az = fmaf(mr3, dz, S.az);
    }
    if (first_j) {
        S.jx = mr3 * jx;
        S.jy = mr3 * jy;
        S.jz = mr3 * jz;
    } else {
        S.jx = fmaf(mr3, jx, S.jx);
        S.jy = fmaf(mr3, jy, S.jy);
        S.jz = fmaf(mr3, jz, S.jz);
    }
}

// Near-field test and parameters of one work item.
struct NearF {
    float near2f;   // FP32 threshold on r^2 + eps^2 (>= eps^2 in FP32)
    double eps2;    // FP64 softening of the near terms
};

// Mixed pair terms.  The FP32 part runs branch-free for every pair, with
// the near pairs' 1/r masked to zero; it returns whether the pair is far
// (not near; a NaN distance counts as far and poisons the FP32 sums).  The
// caller evaluates the (rare) near pairs in FP64 later.
__device__ __forceinline__ bool far_pair(float dx, float dy, float dz, float dvx, float dvy,
                                         float dvz, float eps2f, float near2f, float mj,
                                         bool first, bool first_j, SumF& S)
{
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
    const bool far = !(r2 <= near2f);
    const float ri = far ? rsq_f32(r2) : 0.0f;
    far_terms(dx, dy, dz, dvx, dvy, dvz, ri, mj, first, first_j, S);
    return far;
}

// The near test of a pair, repeated bit for bit after the FP32 pass.
__device__ __forceinline__ bool near_test(float dx, float dy, float dz, float eps2f,
                                          float near2f)
{
    return fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f))) <= near2f;
}

// Cast form: FP64 differences rounded to FP32.
__device__ __forceinline__ bool pair_mixed(const I64& I, float eps2f, float near2f, double xj,
                                           double yj, double zj, double vxj, double vyj,
                                           double vzj, float mj, bool first, SumF& S)
{
    return far_pair((float)(xj - I.x), (float)(yj - I.y), (float)(zj - I.z),
                    (float)(vxj - I.vx), (float)(vyj - I.vy), (float)(vzj - I.vz), eps2f,
                    near2f, mj, first, first, S);
}

__device__ __forceinline__ bool near_mixed_test(const I64& I, float eps2f, float near2f,
                                                double xj, double yj, double zj)
{
    return near_test((float)(xj - I.x), (float)(yj - I.y), (float)(zj - I.z), eps2f, near2f);
}

template <typename RUN>
__device__ __forceinline__ void near_mixed(const I64& I, const NearF& nf, double xj, double yj,
                                           double zj, double vxj, double vyj, double vzj,
                                           double mj, bool self, RUN& R)
{
    double o[7];
    near_terms(xj - I.x, yj - I.y, zj - I.z, vxj - I.vx, vyj - I.vy, vzj - I.vz, mj, nf.eps2,
               self, o);
    add_near(R, o);
}

// Split form of the mixed pair term: every FP64 coordinate c is held as
// hi = fl32(c), lo = fl32(c - hi), and the difference is formed in FP32 as
// (hi_j - hi_i) + (lo_j - lo_i).  When both coordinates share a sign and
// lie within a factor of two the hi difference is exact (Sterbenz) and the
// result carries the one FP32 rounding of the cast form; otherwise (far
// pairs) it may round twice.  Near pairs are rebuilt in FP64 from the
// words (hi + lo holds c to 2^-48 relative).
struct I32S {  // i-particle, split coordinates
    float xh, xl, yh, yl, zh, zl, vxh, vxl, vyh, vyl, vzh, vzl;
};

__device__ __forceinline__ void split(double c, float& h, float& l)
{
    h = (float)c;
    l = (float)(c - (double)h);
}

__device__ __forceinline__ double join_diff(float jh, float jl, float ih, float il)
{
    return ((double)jh - (double)ih) + ((double)jl - (double)il);
}

__device__ __forceinline__ bool pair_split(const I32S& I, float eps2f, float near2f,
                                           const float* J, float mj, bool first, SumF& S)
{
    return far_pair((J[0] - I.xh) + (J[1] - I.xl), (J[2] - I.yh) + (J[3] - I.yl),
                    (J[4] - I.zh) + (J[5] - I.zl), (J[6] - I.vxh) + (J[7] - I.vxl),
                    (J[8] - I.vyh) + (J[9] - I.vyl), (J[10] - I.vzh) + (J[11] - I.vzl), eps2f,
                    near2f, mj, first, first, S);
}

__device__ __forceinline__ bool near_split_test(const I32S& I, float eps2f, float near2f,
                                                const float* J)
{
    return near_test((J[0] - I.xh) + (J[1] - I.xl), (J[2] - I.yh) + (J[3] - I.yl),
                     (J[4] - I.zh) + (J[5] - I.zl), eps2f, near2f);
}

template <typename RUN>
__device__ __forceinline__ void near_split(const I32S& I, const NearF& nf, const float* J,
                                           double mj, bool self, RUN& R)
{
    double o[7];
    near_terms(join_diff(J[0], J[1], I.xh, I.xl), join_diff(J[2], J[3], I.yh, I.yl),
               join_diff(J[4], J[5], I.zh, I.zl), join_diff(J[6], J[7], I.vxh, I.vxl),
               join_diff(J[8], J[9], I.vyh, I.vyl), join_diff(J[10], J[11], I.vzh, I.vzl), mj,
               nf.eps2, self, o);
    add_near(R, o);
}

// Paper-faithful mixed term (Section 3.2 as printed): velocities held in
// FP32 and their difference taken in FP32; everything else as pair_mixed.
// Its near field (radius 0 by default) holds the self pair and coincident
// particles only.
struct I64SP {  // i-particle: FP64 position, FP32 velocity
    double x, y, z;
    float vx, vy, vz;
};

__device__ __forceinline__ bool pair_sp(const I64SP& I, float eps2f, float near2f, double xj,
                                        double yj, double zj, float vxj, float vyj, float vzj,
                                        float mj, bool first, SumF& S)
{
    return far_pair((float)(xj - I.x), (float)(yj - I.y), (float)(zj - I.z), vxj - I.vx,
                    vyj - I.vy, vzj - I.vz, eps2f, near2f, mj, first, false, S);
}

__device__ __forceinline__ bool near_sp_test(const I64SP& I, float eps2f, float near2f,
                                             double xj, double yj, double zj)
{
    return near_test((float)(xj - I.x), (float)(yj - I.y), (float)(zj - I.z), eps2f, near2f);
}

__device__ __forceinline__ void near_sp(const I64SP& I, const NearF& nf, double xj, double yj,
                                        double zj, float vxj, float vyj, float vzj, double mj,
                                        bool self, SumD& R)
{
    double o[7];
    near_terms(xj - I.x, yj - I.y, zj - I.z, (double)vxj - (double)I.vx,
               (double)vyj - (double)I.vy, (double)vzj - (double)I.vz, mj, nf.eps2, self, o);
    add_near(R, o);
}

// Flush of the paper-faithful mode: acceleration and potential runs go to
// the FP64 sums, the jerk stays in its FP32 accumulator (never flushed).
// (No flush clears the run sums: the next run's first term restarts them.)
__device__ __forceinline__ void flush_keep_jerk(const SumF& f, SumD& d)
{
    d.ax += (double)f.ax; d.ay += (double)f.ay; d.az += (double)f.az;
    d.pp += (double)f.pp;
}

// Error estimate of the mixed paths: the squares of each FP32 run sum.
template <typename RUN>
__device__ __forceinline__ void add_estimate(const SumF& f, RUN& d)
{
    d.ea = fmaf(f.ax, f.ax, fmaf(f.ay, f.ay, fmaf(f.az, f.az, d.ea)));
    d.ej = fmaf(f.jx, f.jx, fmaf(f.jy, f.jy, fmaf(f.jz, f.jz, d.ej)));
}

__device__ __forceinline__ void flush(const SumF& f, SumD& d)
{
    add_estimate(f, d);
    d.ax += (double)f.ax; d.ay += (double)f.ay; d.az += (double)f.az;
    d.jx += (double)f.jx; d.jy += (double)f.jy; d.jz += (double)f.jz;
    d.pp += (double)f.pp;
}

__device__ __forceinline__ void flush(const SumF& f, Sum2F& d)
{
    add_estimate(f, d);
    d.ax.add(f.ax); d.ay.add(f.ay); d.az.add(f.az);
    d.jx.add(f.jx); d.jy.add(f.jy); d.jz.add(f.jz);
    d.pp.add(f.pp);
}

// LDS tile of j-particles (SoA), FP64 path.
template <typename MT>
struct Tile {
    double x[kTJ], y[kTJ], z[kTJ], vx[kTJ], vy[kTJ], vz[kTJ];
    MT m[kTJ];
};

// The mixed tiles have kTJPad slots: those past the staged particles hold
// zero-mass particles at 1e30 (finite in FP32, r^2 overflows to +inf, so
// 1/r = 0, the pair adds exactly zero and is never near).  A lane may read
// up to L - 1 slots past a ragged tile's end.
constexpr int kTJPad = kTJ + 64;
constexpr double kFarAway = 1e30;

// FP32 hi and lo words of a mass (hi for the FP32 terms, hi + lo for the
// FP64 near terms), side by side: a tile's per-j records all have an
// 8-byte stride and are addressed from one register.
struct MassHL {
    float hi, lo;
};

// Mixed (cast form): FP64 coordinates and the mass words.
struct TileM {
    double x[kTJPad], y[kTJPad], z[kTJPad], vx[kTJPad], vy[kTJPad], vz[kTJPad];
    MassHL m[kTJPad];
    __device__ void pad(int k)
    {
        x[k] = y[k] = z[k] = kFarAway;
        vx[k] = vy[k] = vz[k] = 0.0;
        m[k] = MassHL{0.0f, 0.0f};
    }
};

// LDS tile of j-particles with split coordinates: c[k][j] for the twelve
// hi/lo words (x, y, z, vx, vy, vz), and the mass words.
struct TileS {
    float c[12][kTJPad];
    float m[kTJPad], mlo[kTJPad];
    __device__ void pad(int k)
    {
#pragma unroll
        for (int w = 0; w < 12; ++w) c[w][k] = (w < 6 && (w & 1) == 0) ? (float)kFarAway : 0.0f;
        m[k] = mlo[k] = 0.0f;
    }
};

// LDS tile for the paper-faithful mode: FP64 positions, FP32 velocities.
struct TileSP {
    double x[kTJPad], y[kTJPad], z[kTJPad];
    float vx[kTJPad], vy[kTJPad], vz[kTJPad], m[kTJPad], mlo[kTJPad];
    __device__ void pad(int k)
    {
        x[k] = y[k] = z[k] = kFarAway;
        vx[k] = vy[k] = vz[k] = 0.0f;
        m[k] = mlo[k] = 0.0f;
    }
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


// Mixed tile loops.  Each lane takes runs of KR of its j (every L-th
// j of the tile).  A run's pair terms are summed in FP32 with no branch and
// no per-lane guard: slots past the tile's end hold zero-mass particles far
// away (see pad_tile), so every lane runs the same trip count, and near
// pairs are masked to zero.  The wave notes in one scalar word which of
// the run's j met a near pair in some lane; after the run those j are
// visited again (rare), the FP32 near test is repeated bit for bit and the
// near pairs are evaluated in FP64 into the running sums.  Then the FP32
// run sums are flushed.
// bit if some lane's ballot bit is clear, else 0.  Scalar instructions only
// (written out because the compiler otherwise moves the wave-uniform
// condition through a vector register and back, two vector instructions
// per j).
__device__ __forceinline__ uint32_t run_hit_bit(uint64_t far_ballot, uint32_t bit)
{
    uint32_t t;
    asm("s_cmp_lg_u64 %1, -1\n\ts_cselect_b32 %0, %2, 0"
        : "=s"(t)
        : "s"(far_ballot), "s"(bit)
        : "scc");
    return t;
}

template <int KR, typename FAR, typename NEARFN, typename FLUSH, typename ZERO>
__device__ __forceinline__ void mixed_runs(int cnt, int sub, int L, FAR far, NEARFN near_fn,
                                           FLUSH flush_fn, ZERO zero_fn)
{
    static_assert(KR >= 1 && KR <= 32, "a run's near hits are one 32-bit word");
    const int step = KR * L;
    for (int jb = 0; jb < cnt; jb += step) {
        const int je = (jb + step < cnt) ? jb + step : cnt;
        const int nk = (je - jb + L - 1) / L;   // j per lane in this run (uniform)
        uint32_t hit = 0;
        // every lane of the wave is active here: far() returns the AND of
        // its particles' ballots of "far", so a lane that met a near pair at
        // its k-th j clears its bit.  (A ballot is a convergent operation,
        // which rules out unrolling a loop of unknown trip count: full runs
        // take the constant-trip form, whose first term starts the run sums.)
        if (nk == KR) {
#pragma unroll
            for (int k = 0; k < KR; ++k)
                hit |= run_hit_bit(far(jb + sub + k * L, k == 0), 1u << k);
        } else {
            zero_fn();
            for (int k = 0; k < nk; ++k)
                hit |= run_hit_bit(far(jb + sub + k * L, false), 1u << k);
        }
        flush_fn();
        while (__builtin_expect(hit != 0, 0)) {
            const int k = __builtin_ctz(hit);
            hit &= hit - 1;
            near_fn(jb + sub + k * L);
        }
    }
}

template <int IPL, int KR, typename RUN>
__device__ __forceinline__ void tile_mixed(const TileM& T, int cnt, int sub, int L, int tb,
                                           const int (&ii)[IPL], const I64 (&I)[IPL],
                                           float eps2f, const NearF& nf, SumF (&f)[IPL],
                                           RUN (&S)[IPL])
{
    mixed_runs<KR>(
        cnt, sub, L,
        [&](int jj, bool first) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const double vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj];
            const float mj = T.m[jj].hi;
            uint64_t fr = ~0ull;
#pragma unroll
            for (int q = 0; q < IPL; ++q)
                fr &= __builtin_amdgcn_ballot_w64(pair_mixed(I[q], eps2f, nf.near2f, xj, yj, zj,
                                                             vxj, vyj, vzj, mj, first, f[q]));
            return fr;
        },
        [&](int jj) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const double vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj];
            const MassHL mw = T.m[jj];
            const double mj = (double)mw.hi + (double)mw.lo;
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                if (near_mixed_test(I[q], eps2f, nf.near2f, xj, yj, zj))
                    near_mixed(I[q], nf, xj, yj, zj, vxj, vyj, vzj, mj, tb + jj == ii[q], S[q]);
                __builtin_amdgcn_sched_barrier(0);   // one particle's FP64 pair at a time
            }
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) flush(f[q], S[q]);
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) f[q].zero();
        });
}

template <int IPL, int KR, typename RUN>
__device__ __forceinline__ void tile_split(const TileS& T, int cnt, int sub, int L, int tb,
                                           const int (&ii)[IPL], const I32S (&I)[IPL],
                                           float eps2f, const NearF& nf, SumF (&f)[IPL],
                                           RUN (&S)[IPL])
{
    mixed_runs<KR>(
        cnt, sub, L,
        [&](int jj, bool first) {
            float J[12];
#pragma unroll
            for (int w = 0; w < 12; ++w) J[w] = T.c[w][jj];
            const float mj = T.m[jj];
            uint64_t fr = ~0ull;
#pragma unroll
            for (int q = 0; q < IPL; ++q)
                fr &= __builtin_amdgcn_ballot_w64(
                    pair_split(I[q], eps2f, nf.near2f, J, mj, first, f[q]));
            return fr;
        },
        [&](int jj) {
            float J[12];
#pragma unroll
            for (int w = 0; w < 12; ++w) J[w] = T.c[w][jj];
            const double mj = (double)T.m[jj] + (double)T.mlo[jj];
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                if (near_split_test(I[q], eps2f, nf.near2f, J))
                    near_split(I[q], nf, J, mj, tb + jj == ii[q], S[q]);
                __builtin_amdgcn_sched_barrier(0);   // one particle's FP64 pair at a time
            }
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) flush(f[q], S[q]);
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) f[q].zero();
        });
}

template <int IPL, int KR>
__device__ __forceinline__ void tile_sp(const TileSP& T, int cnt, int sub, int L, int tb,
                                        const int (&ii)[IPL], const I64SP (&I)[IPL],
                                        float eps2f, const NearF& nf, SumF (&f)[IPL],
                                        SumD (&S)[IPL])
{
    mixed_runs<KR>(
        cnt, sub, L,
        [&](int jj, bool first) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const float vxj = T.vx[jj], vyj = T.vy[jj], vzj = T.vz[jj], mj = T.m[jj];
            uint64_t fr = ~0ull;
#pragma unroll
            for (int q = 0; q < IPL; ++q)
                fr &= __builtin_amdgcn_ballot_w64(pair_sp(I[q], eps2f, nf.near2f, xj, yj, zj,
                                                          vxj, vyj, vzj, mj, first, f[q]));
            return fr;
        },
        [&](int jj) {
            const double xj = T.x[jj], yj = T.y[jj], zj = T.z[jj];
            const double mj = (double)T.m[jj] + (double)T.mlo[jj];
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                if (near_sp_test(I[q], eps2f, nf.near2f, xj, yj, zj))
                    near_sp(I[q], nf, xj, yj, zj, T.vx[jj], T.vy[jj], T.vz[jj], mj,
                            tb + jj == ii[q], S[q]);
                __builtin_amdgcn_sched_barrier(0);   // one particle's FP64 pair at a time
            }
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) flush_keep_jerk(f[q], S[q]);
        },
        [&]() {
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                f[q].ax = f[q].ay = f[q].az = f[q].pp = 0.0f;
            }
        });
}

// One step of the L lanes' butterfly (see lane_partner) for all seven rows,
// both error estimates and, in the paper-faithful mode, the FP32 jerk sums
// of every particle of the lane.
template <int O, int IPL, bool SP>
__device__ __forceinline__ void lanes_sum_step(double (&out)[IPL][kRows], float (&ea)[IPL],
                                               float (&ej)[IPL], float (&fj)[IPL][3])
{
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
#pragma unroll
        for (int r = 0; r < 7; ++r) out[q][r] += lane_partner<O>(out[q][r]);
        ea[q] += lane_partner<O>(ea[q]);
        ej[q] += lane_partner<O>(ej[q]);
        if constexpr (SP) {
#pragma unroll
            for (int r = 0; r < 3; ++r) fj[q][r] += lane_partner<O>(fj[q][r]);
        }
    }
}

// Final per-lane values: acc xyz, jerk xyz, pot (-sum m/r); the error
// estimates are combined separately (they are FP32).
__device__ __forceinline__ void finalize(const SumD& S, double out[kRows])
{
    out[0] = S.ax; out[1] = S.ay; out[2] = S.az;
    out[3] = S.jx; out[4] = S.jy; out[5] = S.jz;
    out[6] = -S.pp;
}

__device__ __forceinline__ void finalize(const Sum2F& S, double out[kRows])
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
// Occupancy hints (waves per SIMD) where they cost no spill: the cast
// two-per-lane forms fit four, the split one with FP64 running sums three;
// the two-float split and fused-selection forms get none.
template <int PREC, int IPL, bool SPLIT, bool SEL>
constexpr int sweep_min_waves()
{
    return SEL || IPL != 2 ? 1
           : (!SPLIT && (PREC == 1 || PREC == 3)) ? 4
           : (SPLIT && PREC == 1) ? 3 : 1;
}

template <int PREC, bool POT_ONLY, int IPL, bool SPLIT, bool SEL = false, int KR = kMixedK>
__global__ void __launch_bounds__(kWG, (sweep_min_waves<PREC, IPL, SPLIT, SEL>()))
sweep_kernel(SweepArgs a)
{
    static_assert(!SEL || !POT_ONLY, "the fused selection is for block steps");
    static_assert(!SPLIT || (PREC == 1 || PREC == 2), "split form is for the mixed modes");
    using MT = typename std::conditional<PREC == 0, double, float>::type;
    using RUN = typename std::conditional<PREC == 2, Sum2F, SumD>::type;
    using TT = typename std::conditional<
        SPLIT, TileS,
        typename std::conditional<
            PREC == 3, TileSP,
            typename std::conditional<PREC == 0, Tile<MT>, TileM>::type>::type>::type;
    constexpr bool kMixed = !POT_ONLY && PREC != 0;
    __shared__ TT T;
    __shared__ int32_t s_ioff[kLdsClusters + 1];
    if constexpr (kMixed) {
        // the slots past a full tile are padding for the whole launch
        for (int k = kTJ + (int)threadIdx.x; k < kTJPad; k += kWG) T.pad(k);
    }

    // item offsets of the clusters in LDS when they fit (the item -> cluster
    // search then costs no global round trips)
    const bool ioff_lds = a.n_clusters > 1 && a.n_clusters <= kLdsClusters;
    if (ioff_lds) {
        for (int k = threadIdx.x; k <= a.n_clusters; k += kWG) s_ioff[k] = a.item_off[k];
        __syncthreads();
    }

    SweepPlan* P = a.plan;
    const int tid = threadIdx.x;
    int na, L, ti, s_max, total, fp64_all = 0;
    int64_t jc, Tpred;
    const int32_t* idx_lds = nullptr;
    if constexpr (SEL) {
        __shared__ int32_t s_idx[kFusedSelMax];
        na = select_in_lds(a.pred_t, a.sel_dt, a.n, a.sel_T_end, s_idx, &Tpred);
        int32_t L_, ti_;
        plan_split_wave(a, na, 1, &L_, &ti_, &jc);
        L = L_;
        ti = ti_;
        s_max = na > 0 ? (int)div_ceil(a.n, jc) : 0;
        total = (int)div_ceil_p2(na, ti) * s_max;
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
                P->fp64_all = 0;
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
        fp64_all = P->fp64_all;
        Tpred = a.pred_x ? *a.pred_T : 0;
    }
    if (na == 0) return;
    // a mixed sweep split over two launches (SweepArgs::kind): a launch with
    // no item of its kind leaves at once (one system is all of one kind; an
    // FP64 block is all FP64; with no small systems only such a block has
    // FP64 items)
    if (a.kind != 0) {
        const bool all64 = fp64_all != 0 || (a.n_clusters == 1 && a.n < a.fp64_below);
        const bool none64 = fp64_all == 0 && (a.n_clusters == 1 ? a.n >= a.fp64_below
                                                                 : a.fp64_below <= 1);
        if ((a.kind == 1 && all64) || (a.kind == 2 && none64)) return;
        if (a.kind == 2 && a.defer_fp64 && fp64_all != 0) return;   // the refine launch's
    }
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
        // mixed near field: pairs with |r| < near_factor * N_c^(-1/3) (and
        // the self pair) are summed in FP64
        NearF nf;
        nf.eps2 = eps2;
        {
            double r2n = eps2;
            if (a.near_factor > 0.0) {
                const double rn = a.near_factor / cbrt((double)(ce - cb));
                r2n = fma(rn, rn, eps2);
            }
            nf.near2f = (float)r2n;    // >= fl32(eps2): the self pair is always near
        }
        // a mixed sweep of an ensemble runs as two launches: this kernel
        // takes the items of one kind only, FP64 for small systems and for
        // small blocks (see SweepArgs::kind)
        if (a.kind != 0 && (fp64_all != 0 || (ce - cb) < a.fp64_below) != (a.kind == 2)) {
            item += (int)gridDim.x;
            continue;
        }

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
                        const double mj = a.m[jg];
                        T.m[tid] = (float)mj;
                        T.mlo[tid] = (float)(mj - (double)(float)mj);
                    } else {
                        T.x[tid] = r[0];
                        T.y[tid] = r[1];
                        T.z[tid] = r[2];
                        T.vx[tid] = w[0];   // rounded to FP32 in the paper-faithful mode
                        T.vy[tid] = w[1];
                        T.vz[tid] = w[2];
                        const double mj = a.m[jg];
                        if constexpr (PREC == 0) {
                            T.m[tid] = mj;
                        } else if constexpr (PREC == 3) {
                            T.m[tid] = (float)mj;
                            T.mlo[tid] = (float)(mj - (double)(float)mj);
                        } else {
                            const float h = (float)mj;
                            T.m[tid] = MassHL{h, (float)(mj - (double)h)};
                        }
                    }
                }
            } else if constexpr (kMixed) {
                T.pad(tid);   // a ragged tile: the rest of it is padding
            }

            __syncthreads();
            if constexpr (POT_ONLY || PREC == 0) {
                // FP64: the self pair is masked by an index compare, only in
                // tiles that hold one of the wave's particles
                bool mine = false;
#pragma unroll
                for (int q = 0; q < IPL; ++q)
                    mine = mine || ((int64_t)ii[q] >= tb && (int64_t)ii[q] < tb + cnt);
                const bool need_mask = __any(mine);
                if constexpr (POT_ONLY) {
                    if (need_mask) tile_pot<true>(T, cnt, sub, L, tb, ii[0], I[0], eps2, S[0]);
                    else           tile_pot<false>(T, cnt, sub, L, tb, ii[0], I[0], eps2, S[0]);
                } else {
                    if (need_mask) tile_f64<true, IPL>(T, cnt, sub, L, tb, ii, I, eps2, S);
                    else           tile_f64<false, IPL>(T, cnt, sub, L, tb, ii, I, eps2, S);
                }
            } else if constexpr (SPLIT) {
                tile_split<IPL, KR>(T, cnt, sub, L, (int)tb, ii, IS, eps2f, nf, F, S);
            } else if constexpr (PREC == 3) {
                tile_sp<IPL, KR>(T, cnt, sub, L, (int)tb, ii, ISP, eps2f, nf, F, S);
            } else {
                tile_mixed<IPL, KR>(T, cnt, sub, L, (int)tb, ii, I, eps2f, nf, F, S);
            }
        }

        // the L lanes of a particle combine their sums by an xor butterfly;
        // every row of every particle of the lane takes each butterfly step
        // together, so a step's cross-lane reads are issued back to back
        // (one row after another, they were a chain of ~170 dependent reads)
        double out[IPL][kRows];
        float ea[IPL], ej[IPL];
        float fj[IPL][3];   // the paper-faithful mode's FP32 jerk sums
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            finalize(S[q], out[q]);
            ea[q] = S[q].ea;
            ej[q] = S[q].ej;
            if constexpr (PREC == 3) {
                // the jerk: one FP32 running sum per lane over every L-th j of
                // the whole range (the plan gives this mode one j-chunk), the
                // L lanes' sums added in FP32 too; near pairs, if any, in FP64
                fj[q][0] = F[q].jx;
                fj[q][1] = F[q].jy;
                fj[q][2] = F[q].jz;
            }
        }
        if (L > 1) lanes_sum_step<1, IPL, PREC == 3>(out, ea, ej, fj);
        if (L > 2) lanes_sum_step<2, IPL, PREC == 3>(out, ea, ej, fj);
        if (L > 4) lanes_sum_step<4, IPL, PREC == 3>(out, ea, ej, fj);
        if (L > 8) lanes_sum_step<8, IPL, PREC == 3>(out, ea, ej, fj);
        if (L > 16) lanes_sum_step<16, IPL, PREC == 3>(out, ea, ej, fj);
        if (L > 32) lanes_sum_step<32, IPL, PREC == 3>(out, ea, ej, fj);
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            out[q][kRows - 1] = pack_est(ea[q], ej[q]);
            if constexpr (PREC == 3) {
#pragma unroll
                for (int r = 0; r < 3; ++r) out[q][3 + r] += (double)fj[q][r];
            }
            if (valid[q] && sub == 0) {
                double* dst = a.partial + (int64_t)k * kRows * na + pp[q];
                if (POT_ONLY) {
                    dst[6 * (int64_t)na] = out[q][6];
                } else {
#pragma unroll
                    for (int r = 0; r < kRows; ++r) dst[r * (int64_t)na] = out[q][r];
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
__device__ __forceinline__ void store_reduced(const SweepArgs& a, int p, const double s[kRows])
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
            double s[kRows];
            reduce_partials(a, na, p, s);
            store_reduced<POT_ONLY>(a, p, s);
        }
    } else {
        const int lane = threadIdx.x & 63;
        const int wpb = kWG / 64;
        for (int p = blockIdx.x * wpb + (int)(threadIdx.x >> 6); p < na; p += gridDim.x * wpb) {
            double s[kRows];
            reduce_partials_wave(a, na, p, lane, s);
            if (lane == 0) store_reduced<POT_ONLY>(a, p, s);
        }
    }
}

// The reduce of a mixed sweep with refinement: stores every particle's
// mixed sums and compacts, per unit (a round of a workgroup), the
// positions whose error estimate is too large; refine_plan_kernel then
// lists them and plans the FP64 refine sweep.  Rounds run with uniform
// trip counts over the workgroup (the compaction synchronises it).
__global__ void __launch_bounds__(kWG) reduce_flag_kernel(SweepArgs a)
{
    if (a.defer_fp64 && a.plan->fp64_all) return;
    const int na = a.plan->n_act;
    if (thread_reduce(a.plan->s_max, na)) {
        for (int u = blockIdx.x; u * kWG < na; u += gridDim.x) {
            const int base = u * kWG;
            const int p = base + (int)threadIdx.x;
            bool flag = false;
            if (p < na) {
                double s[kRows];
                reduce_partials(a, na, p, s);
                store_reduced<false>(a, p, s);
                flag = needs_refine(a, s);
            }
            flag_unit(a, u, base, p, p < na, flag);
        }
    } else {
        const int lane = threadIdx.x & 63;
        const int wpb = kWG / 64;
        for (int u = blockIdx.x; u * wpb < na; u += gridDim.x) {
            const int base = u * wpb;
            const int p = base + (int)(threadIdx.x >> 6);
            bool flag = false;
            if (p < na) {
                double s[kRows];
                reduce_partials_wave(a, na, p, lane, s);
                if (lane == 0) store_reduced<false>(a, p, s);
                flag = needs_refine(a, s);
            }
            flag_unit(a, u, base, p, p < na && lane == 0, flag);
        }
    }
}

// One workgroup: the refine list and the plan of the refine sweep ra.
__global__ void __launch_bounds__(kWG) refine_plan_kernel(SweepArgs a, SweepArgs ra)
{
    if (a.defer_fp64 && a.plan->fp64_all) {
        // an FP64 block: the refine sweep takes all of it, in list order
        // (its clusters' runs where the sweep's are)
        const int na = a.plan->n_act;
        for (int k = threadIdx.x; k < na; k += kWG) {
            a.ref_idx[k] = a.idx ? a.idx[k] : k;
            a.ref_p[k] = k;
        }
        if (a.n_clusters > 1)
            for (int c = threadIdx.x; c < a.n_clusters; c += kWG) ra.act_start[c] = a.act_start[c];
        __syncthreads();   // act_start complete before the plan reads it
        plan_body(ra, na);
        return;
    }
    const int na = a.plan->n_act;
    const int unit = thread_reduce(a.plan->s_max, na) ? kWG : kWG / 64;
    const int32_t cnt = build_refine_list(a, ra, na, unit);
    if (threadIdx.x == 0 && a.counters && cnt > 0)
        atomicAdd((unsigned long long*)&a.counters[5], (unsigned long long)cnt);
}

// Writes the refined sums of the flagged particles over their mixed ones
// (a wave per particle: the refine sweep splits j into many chunks); for a
// block the plan put in FP64 these are all of its particles.
__global__ void __launch_bounds__(kWG) refine_scatter_kernel(SweepArgs a, SweepArgs ra)
{
    const int cnt = ra.plan->n_act;
    const int lane = threadIdx.x & 63;
    const int wpb = kWG / 64;
    for (int k = blockIdx.x * wpb + (int)(threadIdx.x >> 6); k < cnt; k += gridDim.x * wpb) {
        double s[kRows];
        reduce_partials_wave(ra, cnt, k, lane, s);
        if (lane == 0) store_reduced<false>(a, a.ref_p[k], s);
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
// differences (MIXED and MIXED_2F only; FP64 and MIXED_SP ignore it); bit 2
// -> FP32 runs of kMixedKLong (the mixed precisions; FP64 ignores it).
template <int PREC, int IPL, bool SPLIT>
SweepFn mixed_fn(bool long_runs)
{
    return long_runs ? sweep_kernel<PREC, false, IPL, SPLIT, false, kMixedKLong>
                     : sweep_kernel<PREC, false, IPL, SPLIT, false, kMixedK>;
}

SweepFn sweep_fn(int precision, int variant, bool pot_only)
{
    if (pot_only) return sweep_kernel<0, true, 1, false>;
    const bool two = (variant & 1) != 0;
    const bool spl = (variant & 2) != 0;
    const bool lng = (variant & 4) != 0;
    if (precision == 0)
        return two ? sweep_kernel<0, false, 2, false> : sweep_kernel<0, false, 1, false>;
    if (precision == 1) {
        if (spl) return two ? mixed_fn<1, 2, true>(lng) : mixed_fn<1, 1, true>(lng);
        return two ? mixed_fn<1, 2, false>(lng) : mixed_fn<1, 1, false>(lng);
    }
    if (precision == 3) return two ? mixed_fn<3, 2, false>(lng) : mixed_fn<3, 1, false>(lng);
    if (spl) return two ? mixed_fn<2, 2, true>(lng) : mixed_fn<2, 1, true>(lng);
    return two ? mixed_fn<2, 2, false>(lng) : mixed_fn<2, 1, false>(lng);
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

// Launches the sweep kernel(s) of one force sweep.  The mixed precisions
// sweep systems of fewer than fp64_below particles in FP64 (at those sizes
// the FP64 sweep is as fast as the FP32 one with its near field, and
// exact): a single system takes one kernel or the other, and an ensemble
// whose cluster sizes straddle the threshold takes both, each kernel doing
// the work items of its kind of cluster.  Both kernels share the plan,
// which fixes the active particles per lane: the FP64 kernel is the
// instantiation with the mixed variant's count.
void launch_sweep_kernels(SweepArgs a, int precision, int variant, int grid, bool pot_only,
                          bool sel, hipStream_t st)
{
    a.ipl = (!pot_only && (variant & 1)) ? 2 : 1;
    auto go = [&](int prec, int kind) {
        a.kind = kind;
        SweepFn f = sel ? sweep_sel_fn(prec, variant) : sweep_fn(prec, variant, pot_only);
        hipLaunchKernelGGL(f, dim3(grid), dim3(kWG), 0, st, a);
    };
    const bool mixed = !pot_only && (precision == 1 || precision == 2);
    const bool straddle = a.n_clusters > 1 && a.fp64_below > 1;
    if (!mixed) {
        go(precision, 0);
    } else if (a.n_cmax < a.fp64_below) {
        go(0, 0);                          // every system is small
    } else if (straddle || (!sel && a.fp64_inter_below > 0)) {
        // the plan decides on the device, per block, which items are FP64;
        // in a block step the refine sweep's launch takes an FP64 block, so
        // only small systems need an FP64 launch here
        go(precision, 1);
        if (straddle || !a.defer_fp64) go(0, 2);
    } else {
        go(precision, 0);                  // no item is
    }
}

hipError_t launch_select_sweep(const SweepArgs& a, int precision, int variant, int grid,
                               hipStream_t st)
{
    launch_sweep_kernels(a, precision, variant, grid, false, true, st);
    return hipGetLastError();
}

hipError_t launch_sweep_only(const SweepArgs& a, int precision, int variant, int grid,
                             hipStream_t st)
{
    launch_sweep_kernels(a, precision, variant, grid, false, false, st);
    return hipGetLastError();
}

// Flagging reduce and FP64 refine sweep (both launch forms).
hipError_t launch_reduce_refine(const SweepArgs& a_in, const SweepArgs& ra_in, int variant,
                                int grid, hipStream_t st)
{
    SweepArgs a = a_in, ra = ra_in;
    a.ipl = ra.ipl = (variant & 1) ? 2 : 1;
    hipLaunchKernelGGL(reduce_flag_kernel, dim3(reduce_grid(a.n_act_max)), dim3(kWG), 0, st, a);
    hipLaunchKernelGGL(refine_plan_kernel, dim3(1), dim3(kWG), 0, st, a, ra);
    // the FP64 kernel with the mixed variant's particles per lane (the plan
    // was made for that count)
    launch_sweep_kernels(ra, 0, variant & 1, grid, false, false, st);
    return hipGetLastError();
}

hipError_t launch_force(const SweepArgs& a_in, const SweepArgs* ra, int precision, int variant,
                        int grid, bool pot_only, hipStream_t st, const hipEvent_t* marks)
{
    SweepArgs a = a_in;
    a.ipl = (!pot_only && (variant & 1)) ? 2 : 1;
    // with refinement, a block the plan puts in FP64 is swept by the refine
    // sweep's launch (the whole block as its list) and scattered from there
    a.defer_fp64 = (!pot_only && ra && a.refine) ? 1 : 0;
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kWG), 0, st, a);
    if (marks) {
        const hipError_t e = hipEventRecord(marks[0], st);
        if (e != hipSuccess) return e;
    }
    launch_sweep_kernels(a, precision, variant, grid, pot_only, false, st);
    if (marks) {
        const hipError_t e = hipEventRecord(marks[1], st);
        if (e != hipSuccess) return e;
    }
    const int rgrid = reduce_grid(a.n_act_max);
    if (pot_only) {
        hipLaunchKernelGGL(reduce_kernel<true>, dim3(rgrid), dim3(kWG), 0, st, a);
    } else if (ra && a.refine) {
        const hipError_t e = launch_reduce_refine(a, *ra, variant, grid, st);
        if (e != hipSuccess) return e;
        SweepArgs r = *ra;
        r.ipl = a.ipl;
        hipLaunchKernelGGL(refine_scatter_kernel, dim3(rgrid), dim3(kWG), 0, st, a, r);
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
