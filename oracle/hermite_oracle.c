/*
 * Plain FP64 CPU oracle for the fourth-order Hermite scheme with block
 * (power-of-two) individual timesteps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the GPU
 * path.
 *
 * It is deliberately slow and literal:
 *   - every floating-point operation is IEEE binary64, round to nearest,
 *     built with -O2 -ffp-contract=off and without -ffast-math;
 *   - sums over j run in ascending j and use Neumaier compensated
 *     summation, so the oracle's own rounding stays far below the 1e-13
 *     tolerance the GPU FP64 path is held to;
 *   - OpenMP splits only the outer loop over i; the j order never changes,
 *     so results do not depend on the thread count.
 *
 * Paper: Tanikawa, Yoshikawa, Okamoto & Nitadori, "N-body simulation for
 * self-gravitating collisional systems with a new SIMD instruction set
 * extension to the x86 architecture, Advanced Vector eXtensions"
 * (arXiv:1104.2700).  Each function cites the section/equation it follows.
 *
 * Layout: every vector field is SoA, [3][n] contiguous (all x, then all y,
 * then all z).  Times are int64 ticks of 2^-tick_bits.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Neumaier compensated sum (Neumaier 1974).                            */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum* a, double t)
{
    double u = a->s + t;
    if (fabs(a->s) >= fabs(t)) a->c += (a->s - u) + t;
    else                       a->c += (t - u) + a->s;
    a->s = u;
}
static inline double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Section 2, equations (acc), (jrk), (pot): softened acceleration,    */
/* jerk and potential of particle i from every j != i (G = 1).         */
/*                                                                    */
/* r_ij = r_j - r_i, v_ij = v_j - v_i, s = r_ij^2 + eps^2,             */
/*   a_i   +=  m_j r_ij / s^{3/2}                                      */
/*   jrk_i +=  m_j / s^{3/2} [ v_ij - 3 (r_ij . v_ij) / s  r_ij ]      */
/*   phi_i -=  m_j / s^{1/2}                                           */
/*                                                                    */
/* The sum runs over j in [j_begin, j_end), skipping j == idx[k]       */
/* (the self term is excluded by index, not by value).                 */
/* cond (optional, [3][n_act]) receives the absolute sums              */
/* sum_j |a_ij|, sum_j |jrk_ij|, sum_j |phi_ij| used for the           */
/* cancellation-aware tolerance.                                       */
/* ------------------------------------------------------------------ */
void oracle_force(int64_t n, const double* pos, const double* vel,
                  const double* m, int64_t n_act, const int32_t* idx,
                  double eps2, int64_t j_begin, int64_t j_end,
                  double* acc, double* jrk, double* pot, double* cond)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    const double *vx = vel, *vy = vel + n, *vz = vel + 2 * n;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < n_act; ++k) {
        const int64_t i = idx[k];
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        nsum jx = {0, 0}, jy = {0, 0}, jz = {0, 0};
        nsum ph = {0, 0};
        double abs_a = 0.0, abs_j = 0.0, abs_p = 0.0;
        for (int64_t j = j_begin; j < j_end; ++j) {
            if (j == i) continue;
            const double rx = x[j] - x[i];
            const double ry = y[j] - y[i];
            const double rz = z[j] - z[i];
            const double wx = vx[j] - vx[i];
            const double wy = vy[j] - vy[i];
            const double wz = vz[j] - vz[i];
            const double s = rx * rx + ry * ry + rz * rz + eps2;
            const double q = 1.0 / sqrt(s);          /* 1 / s^{1/2} */
            const double mq3 = m[j] * (q * q * q);   /* m_j / s^{3/2} */
            const double rv = rx * wx + ry * wy + rz * wz;
            const double c3 = 3.0 * rv / s;          /* 3 (r.v) / s */
            const double tax = mq3 * rx, tay = mq3 * ry, taz = mq3 * rz;
            const double tjx = mq3 * (wx - c3 * rx);
            const double tjy = mq3 * (wy - c3 * ry);
            const double tjz = mq3 * (wz - c3 * rz);
            const double tph = -(m[j] * q);
            nsum_add(&ax, tax); nsum_add(&ay, tay); nsum_add(&az, taz);
            nsum_add(&jx, tjx); nsum_add(&jy, tjy); nsum_add(&jz, tjz);
            nsum_add(&ph, tph);
            abs_a += sqrt(tax * tax + tay * tay + taz * taz);
            abs_j += sqrt(tjx * tjx + tjy * tjy + tjz * tjz);
            abs_p += fabs(tph);
        }
        acc[k] = nsum_get(&ax);
        acc[n_act + k] = nsum_get(&ay);
        acc[2 * n_act + k] = nsum_get(&az);
        jrk[k] = nsum_get(&jx);
        jrk[n_act + k] = nsum_get(&jy);
        jrk[2 * n_act + k] = nsum_get(&jz);
        pot[k] = nsum_get(&ph);
        if (cond) {
            cond[k] = abs_a;
            cond[n_act + k] = abs_j;
            cond[2 * n_act + k] = abs_p;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Section 2, equations (xpred), (vpred): Taylor predictor.            */
/* dt = (T - t_i) * 2^-tick_bits is exact in binary64 (an integer      */
/* below 2^53 times a power of two).  Applied to every particle.       */
/* ------------------------------------------------------------------ */
void oracle_predict(int64_t n, const double* pos, const double* vel,
                    const double* acc, const double* jrk, const int64_t* t,
                    int64_t T, int tick_bits, double* xp, double* vp)
{
    const double tick = ldexp(1.0, -tick_bits);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const double dt = (double)(T - t[i]) * tick;
        for (int d = 0; d < 3; ++d) {
            const int64_t o = d * n + i;
            xp[o] = pos[o] + vel[o] * dt + acc[o] / 2.0 * (dt * dt)
                  + jrk[o] / 6.0 * (dt * dt * dt);
            vp[o] = vel[o] + acc[o] * dt + jrk[o] / 2.0 * (dt * dt);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Block selection (Section 2, procedure step 1): the next block time  */
/* is T = min_i (t_i + dt_i); the active particles are those with      */
/* t_i + dt_i == T, listed in ascending index order.                   */
/* Returns n_act.                                                      */
/* ------------------------------------------------------------------ */
int64_t oracle_select(int64_t n, const int64_t* t, const int64_t* dt,
                      int64_t* T_out, int32_t* idx)
{
    int64_t T = INT64_MAX;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] < T) T = t[i] + dt[i];
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] == T) idx[k++] = (int32_t)i;
    *T_out = T;
    return k;
}

static double norm3(double a, double b, double c)
{
    return sqrt(a * a + b * b + c * c);
}

/* ------------------------------------------------------------------ */
/* Section 2, equation (timestep): the Aarseth criterion, then the     */
/* power-of-two quantisation of the hierarchical scheme.               */
/*                                                                    */
/*   R = (|a||s| + |j|^2) / (|j||c| + |s|^2)                           */
/*   form 0 ("as printed"): dt_crit = eta * sqrt(R)                    */
/*   form 1 (classic):      dt_crit = sqrt(eta * R)                    */
/*                                                                    */
/* The paper prints eta outside the square root; form 1 is the usual   */
/* Aarseth form.  Quantisation: the largest 2^-k <= dt_crit, clamped   */
/* to k in [k_min, k_max]; at most double the previous step            */
/* (k >= k_old - 1, skipped when k_old < 0); then halved until the     */
/* block time T is a multiple of it.  A criterion that is NaN or       */
/* +inf (no force, no jerk) maps to k_min; a step forced to k_max      */
/* while the criterion asked for less sets *clamped.                   */
/* Returns dt in ticks.                                                */
/* ------------------------------------------------------------------ */
double oracle_aarseth(const double a[3], const double j[3], const double s[3],
                      const double c[3], double eta, int form)
{
    const double A = norm3(a[0], a[1], a[2]);
    const double J = norm3(j[0], j[1], j[2]);
    const double S = norm3(s[0], s[1], s[2]);
    const double C = norm3(c[0], c[1], c[2]);
    const double R = (A * S + J * J) / (J * C + S * S);
    return form == 0 ? eta * sqrt(R) : sqrt(eta * R);
}

int64_t oracle_quantize(double dt_crit, int k_old, int64_t T, int tick_bits,
                        int k_min, int k_max, int* k_out, int* clamped)
{
    int k;
    *clamped = 0;
    if (!(dt_crit == dt_crit) || dt_crit == INFINITY) {
        k = k_min;
    } else if (dt_crit <= 0.0) {
        k = k_max;
        *clamped = 1;
    } else {
        int e;
        frexp(dt_crit, &e);          /* dt_crit = f 2^e, f in [1/2, 1) */
        k = 1 - e;                   /* 2^(e-1) <= dt_crit < 2^e       */
        if (k < k_min) k = k_min;
        if (k > k_max) { k = k_max; *clamped = 1; }
    }
    if (k_old >= 0 && k < k_old - 1) k = k_old - 1;
    while (k < k_max && (T & ((((int64_t)1) << (tick_bits - k)) - 1)) != 0)
        ++k;
    *k_out = k;
    return ((int64_t)1) << (tick_bits - k);
}

static int ticks_to_k(int64_t dt, int tick_bits)
{
    int k = tick_bits;
    while (dt > 1) { dt >>= 1; --k; }
    return k;
}

/* ------------------------------------------------------------------ */
/* Section 2, snap/crackle and corrector equations, then procedure     */
/* steps 5-8.  For each active i (dt = dt_i, the step just taken):     */
/*   s0 = 2 [-3 (a0 - a1) - (2 j0 + j1) dt] / dt^2                     */
/*   c0 = 6 [ 2 (a0 - a1) + (j0 + j1) dt] / dt^3                       */
/*   r1 = rp + s0 dt^4 / 24 + c0 dt^5 / 120                            */
/*   v1 = vp + s0 dt^3 / 6  + c0 dt^4 / 24                             */
/* then a0 <- a1, j0 <- j1, t_i <- T, and the next step comes from the */
/* criterion evaluated at the new time with s1 = s0 + c0 dt, c1 = c0.  */
/* acc1/jrk1/pot1 are compact [3][n_act] / [n_act] outputs of the      */
/* force sweep.  crit_out (optional, [n_act]) receives the criterion   */
/* value before quantisation.  Returns the number of clamped steps.    */
/* ------------------------------------------------------------------ */
int64_t oracle_correct(int64_t n, int64_t n_act, const int32_t* idx,
                       int64_t T, int tick_bits,
                       const double* xp, const double* vp,
                       const double* acc1, const double* jrk1,
                       const double* pot1,
                       double* pos, double* vel, double* acc, double* jrk,
                       double* pot, int64_t* t, int64_t* dt,
                       double eta, int form, int k_min, int k_max,
                       double* crit_out)
{
    int64_t n_clamped = 0;
    const double tick = ldexp(1.0, -tick_bits);
    for (int64_t k = 0; k < n_act; ++k) {
        const int64_t i = idx[k];
        const double h = (double)dt[i] * tick;
        double s1[3], c0v[3], a1v[3], j1v[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t o = d * n + i;
            const double a0 = acc[o], j0 = jrk[o];
            const double a1 = acc1[d * n_act + k], j1 = jrk1[d * n_act + k];
            const double s0 = 2.0 * (-3.0 * (a0 - a1) - (2.0 * j0 + j1) * h)
                            / (h * h);
            const double c0 = 6.0 * (2.0 * (a0 - a1) + (j0 + j1) * h)
                            / (h * h * h);
            pos[o] = xp[o] + s0 / 24.0 * (h * h * h * h)
                   + c0 / 120.0 * (h * h * h * h * h);
            vel[o] = vp[o] + s0 / 6.0 * (h * h * h)
                   + c0 / 24.0 * (h * h * h * h);
            acc[o] = a1;
            jrk[o] = j1;
            s1[d] = s0 + c0 * h;
            c0v[d] = c0;
            a1v[d] = a1;
            j1v[d] = j1;
        }
        pot[i] = pot1[k];
        t[i] = T;
        const double crit = oracle_aarseth(a1v, j1v, s1, c0v, eta, form);
        if (crit_out) crit_out[k] = crit;
        int knew, cl;
        dt[i] = oracle_quantize(crit, ticks_to_k(dt[i], tick_bits), T,
                                tick_bits, k_min, k_max, &knew, &cl);
        n_clamped += cl;
    }
    return n_clamped;
}

/* ------------------------------------------------------------------ */
/* First step (the paper gives none; reading: dt0 = eta_f |a| / |j|    */
/* with eta_f = eta (form 0) or sqrt(eta) (form 1), quantised with     */
/* T = 0 and no growth limit).  eta_init > 0 replaces eta_f: |a|/|j|   */
/* has no guard against a small initial jerk, and a smaller start-up   */
/* factor keeps the first step from dominating a run's energy error.   */
/* Sets t_i = 0.                                                       */
/* ------------------------------------------------------------------ */
int64_t oracle_init_dt(int64_t n, const double* acc, const double* jrk,
                       int64_t* t, int64_t* dt, int tick_bits,
                       double eta, int form, double eta_init, int k_min, int k_max)
{
    int64_t n_clamped = 0;
    const double eta_f = form == 0 ? eta : sqrt(eta);
    const double eta_s = eta_init > 0.0 ? eta_init : eta_f;
    for (int64_t i = 0; i < n; ++i) {
        const double A = norm3(acc[i], acc[n + i], acc[2 * n + i]);
        const double J = norm3(jrk[i], jrk[n + i], jrk[2 * n + i]);
        const double crit = eta_s * A / J;
        int k, cl;
        t[i] = 0;
        dt[i] = oracle_quantize(crit, -1, 0, tick_bits, k_min, k_max, &k, &cl);
        n_clamped += cl;
    }
    return n_clamped;
}

/* ------------------------------------------------------------------ */
/* Energy check (Section 2 after eq. (pot), Section 4): E = K + W with */
/* K = 1/2 sum m v^2 and W = 1/2 sum m_i phi_i, phi from a separate    */
/* FP64 sweep at the (synchronised, corrected) positions.              */
/* ------------------------------------------------------------------ */
void oracle_energy(int64_t n, const double* pos, const double* vel,
                   const double* m, double eps2, double* K, double* W,
                   double* phi_scratch, int32_t* idx_scratch,
                   double* acc_scratch, double* jrk_scratch)
{
    for (int64_t i = 0; i < n; ++i) idx_scratch[i] = (int32_t)i;
    oracle_force(n, pos, vel, m, n, idx_scratch, eps2, 0, n,
                 acc_scratch, jrk_scratch, phi_scratch, NULL);
    nsum k = {0, 0}, w = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double v2 = vel[i] * vel[i] + vel[n + i] * vel[n + i]
                        + vel[2 * n + i] * vel[2 * n + i];
        nsum_add(&k, 0.5 * m[i] * v2);
        nsum_add(&w, 0.5 * m[i] * phi_scratch[i]);
    }
    *K = nsum_get(&k);
    *W = nsum_get(&w);
}

/* ------------------------------------------------------------------ */
/* Thread count of the parallel loops (timing only; results do not     */
/* depend on it).  n < 1 leaves it unchanged.  Returns the count now   */
/* in effect.                                                          */
/* ------------------------------------------------------------------ */
int oracle_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
