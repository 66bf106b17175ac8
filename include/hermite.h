/*
 * hermite.h -- C ABI of libhermite, an MI355X (gfx950) implementation of the
 * hot path of the fourth-order Hermite N-body scheme with block
 * (power-of-two individual) timesteps of Tanikawa, Yoshikawa, Okamoto &
 * Nitadori (arXiv:1104.2700):
 *
 *   select the block  ->  predict  ->  force/jerk/potential sweep  ->
 *   correct + new timestep        (Section 2, procedure steps 1-8)
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Every function returns int: HERMITE_OK (0) or a negative error code;
 *    hermite_last_error() then returns a thread-local message.  Nothing
 *    throws across the ABI.
 *  - "device" pointers are HIP device memory (e.g. torch tensors on cuda:0,
 *    data_ptr()), owned by the caller.  The library never frees them.  The
 *    library owns only its context scratch (allocated on first need and
 *    freed by hermite_destroy).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue work and return without synchronising, unless stated.
 *    Errors of kernels that run later surface at the next synchronising
 *    call (hermite_sync, hermite_counters, hermite_run).
 *  - Vector fields are SoA: a pointer to 3*n doubles laid out [3][n]
 *    (all x, then all y, then all z).  Compact per-active outputs are
 *    [3][stride] with stride = n_act_max.
 *  - Times are int64 ticks of 2^-tick_bits; the global time unit is 1.
 *  - G = 1 (standard N-body units, Section 4).
 *  - Index lists are int32, ascending, without duplicates.  Violations are
 *    undefined behaviour (not checked on the device).
 *  - A context is not thread-safe: use one per host thread.
 */
#ifndef HERMITE_H
#define HERMITE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define HERMITE_OK          0
#define HERMITE_EINVAL     -1  /* bad argument (null, size, range, NaN)   */
#define HERMITE_ENODEV     -2  /* no such HIP device                      */
#define HERMITE_EHIP       -3  /* a HIP runtime call failed (message set) */
#define HERMITE_ENOMEM     -4  /* scratch allocation failed               */
#define HERMITE_ENONFINITE -5  /* non-finite state detected (see          */
                               /* hermite_check_finite, hermite_run)      */
#define HERMITE_ENOTSUP    -6  /* reserved; not returned by this version  */

/* ---- precision of the force/jerk sweep -------------------------------- */
/* FP64 everywhere.                                                        */
#define HERMITE_FP64      0
/* Section 3.2 precision split, modified: relative position and velocity  */
/* subtracted in FP64, cast to FP32 for the pair arithmetic (r^2 + eps^2, */
/* rsqrt, jerk and potential terms), partial sums over short runs of j in */
/* FP32 and the running sums of acc, jerk and pot in FP64.  Near pairs,   */
/* and small systems altogether, are evaluated in FP64 (see              */
/* hermite_set_mixed_policy).                                             */
#define HERMITE_MIXED     1
/* As HERMITE_MIXED, but the running sums are two-float (FP32 hi + lo,    */
/* compensated by TwoSum) instead of FP64.                                */
#define HERMITE_MIXED_2F  2
/* Section 3.2 precision split as printed: FP64 relative position, FP32   */
/* velocities and FP32 velocity difference, FP32 pair arithmetic, FP64    */
/* sums of acc and pot, and the jerk summed in FP32: one running sum per  */
/* lane over every L-th j of the whole system (no j-split across work     */
/* items in this mode), the L lanes' sums added in FP32.                  */
#define HERMITE_MIXED_SP  3

/* ---- timestep criterion forms (Section 2, eq. (timestep)) ------------ */
#define HERMITE_DT_PAPER    0  /* dt = eta * sqrt(R), as printed          */
#define HERMITE_DT_AARSETH  1  /* dt = sqrt(eta * R), the classic form    */

/* Particle state.  All pointers are device pointers, caller-owned.
 * tick_bits in [1, 52]; k_max of the timestep parameters <= tick_bits. */
typedef struct hermite_state {
    int64_t n;            /* number of particles, 1 <= n <= INT32_MAX     */
    int32_t tick_bits;    /* time tick = 2^-tick_bits                     */
    int32_t reserved0;
    const double* m;      /* [n] masses                                   */
    double* x;            /* [3][n] positions at t_i                      */
    double* v;            /* [3][n] velocities at t_i                     */
    double* a;            /* [3][n] accelerations a0 at t_i               */
    double* j;            /* [3][n] jerks j0 at t_i                       */
    double* xp;           /* [3][n] predicted positions (written)         */
    double* vp;           /* [3][n] predicted velocities (written)        */
    double* pot;          /* [n] potential at t_i (written by correct)    */
    int64_t* t;           /* [n] last time of each particle, in ticks     */
    int64_t* dt;          /* [n] current step of each particle, in ticks  */
} hermite_state;

/* Aarseth criterion and quantisation (Section 2, eq. (timestep) and the
 * hierarchical power-of-two scheme).  Steps are 2^-k, k in [k_min, k_max],
 * at most double the previous step, commensurate with the block time. */
typedef struct hermite_dt_params {
    double  eta;          /* accuracy parameter, > 0                      */
    int32_t form;         /* HERMITE_DT_PAPER or HERMITE_DT_AARSETH       */
    int32_t k_min;        /* largest step 2^-k_min, k_min >= 0            */
    int32_t k_max;        /* smallest step 2^-k_max, k_max <= tick_bits   */
    int32_t reserved0;
    double  eta_init;     /* start-up factor of hermite_init_dt; 0 selects */
                          /* the steady factor, else > 0                   */
} hermite_dt_params;

/* Independent clusters in one state (ensembles).  Particles of cluster c
 * occupy [offsets[c], offsets[c+1]); a particle feels only its own
 * cluster, softened by eps2[c].  Both arrays are device memory.  NULL in
 * place of a hermite_clusters* means one system of all n particles. */
typedef struct hermite_clusters {
    int32_t n_clusters;       /* C >= 1                                   */
    int32_t reserved0;
    int64_t max_size;         /* host value: max_c (offsets[c+1]-offsets[c]) */
    const int64_t* offsets;   /* [C+1], offsets[0] = 0, offsets[C] = n,   */
                              /* strictly increasing                      */
    const double* eps2;       /* [C] squared softening per cluster        */
} hermite_clusters;

/* Launch shape of the sweep; see hermite_autotune. */
typedef struct hermite_tuning {
    int32_t target_lanes;     /* lanes the j-split aims to keep busy      */
    int32_t wg_per_cu;        /* persistent workgroups per compute unit   */
    int32_t min_j_per_lane;   /* smallest j-run a lane is given per chunk */
    int32_t variant;          /* inner loop, 0..7: bit 0 = two active     */
                              /* particles per lane; bit 1 = FP32 hi/lo   */
                              /* split differences (MIXED, MIXED_2F only);*/
                              /* bit 2 = FP32 runs of 32 terms instead of */
                              /* 16 between FP64 flushes (mixed modes)    */
} hermite_tuning;

typedef struct hermite_ctx hermite_ctx;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device` (makes it current).
 * ENODEV if the device does not exist. */
int hermite_create(int device, hermite_ctx** out);

/* Free the context's scratch, graphs and streams.  NULL is a no-op. */
int hermite_destroy(hermite_ctx* ctx);

/* Thread-local message of the last error (never NULL). */
const char* hermite_last_error(void);

/* Block until all work the library enqueued on `stream` has finished;
 * reports errors of earlier kernels (EHIP). */
int hermite_sync(hermite_ctx* ctx, void* stream);

/* ---- the hot path -------------------------------------------------------- */

/* Procedure step 1 (Section 2): T = min_i (t_i + dt_i), the active list
 * {i : t_i + dt_i == T} in ascending order.  Outputs stay on the device:
 * idx_out [n] (first n_act entries valid), *n_act_dev, *T_dev.  If
 * T > T_end, *n_act_dev = 0 (nothing to do) and *T_dev still holds T.
 * Pass T_end = INT64_MAX for no limit. */
int hermite_select_block(hermite_ctx* ctx, const hermite_state* s,
                         int32_t* idx_out, int32_t* n_act_dev, int64_t* T_dev,
                         int64_t T_end, void* stream);

/* Procedure steps 2-3, equations (xpred), (vpred): for every particle,
 * with dt_i = (T - t_i) ticks, writes s->xp, s->vp.  T is read from
 * T_dev (device) when non-NULL, else T_host is used.  If n_act_dev is
 * non-NULL and *n_act_dev == 0 the kernel does nothing. */
int hermite_predict(hermite_ctx* ctx, const hermite_state* s,
                    const int64_t* T_dev, int64_t T_host,
                    const int32_t* n_act_dev, void* stream);

/* Procedure step 4, equations (acc), (jrk), (pot): for each active i in
 * idx[0..n_act), sums over every j != i of its system (all n, or its
 * cluster) at the predicted state s->xp, s->vp with softening eps2 (or
 * cl->eps2[c]):
 *     acc  += m_j r / s^{3/2}
 *     jerk += m_j / s^{3/2} (v - 3 (r.v)/s r)
 *     pot  -= m_j / s^{1/2}
 * with r = xp_j - xp_i, v = vp_j - vp_i, s = r^2 + eps2.
 * idx: device [n_act_max], or NULL for the identity (requires
 * n_act_max == n).  n_act_dev: device count, or NULL for n_act_max.
 * Outputs (device): acc [3][n_act_max], jerk [3][n_act_max],
 * pot [n_act_max] (may be NULL); only the first n_act columns written.
 * precision: HERMITE_FP64 / HERMITE_MIXED / HERMITE_MIXED_2F /
 * HERMITE_MIXED_SP.
 * Results are bitwise reproducible run to run for a fixed tuning. */
int hermite_force_jerk(hermite_ctx* ctx, const hermite_state* s,
                       const hermite_clusters* cl,
                       const int32_t* idx, const int32_t* n_act_dev,
                       int32_t n_act_max, double eps2, int precision,
                       double* acc, double* jerk, double* pot, void* stream);

/* Profiling form of hermite_force_jerk (Section 5's per-interaction
 * speed): the same sweep run reps times over the first n_act entries of idx
 * (or all particles, idx NULL and n_act == n), each time bracketed by HIP
 * events on the given stream, waiting for each run to end.  ms_out (host,
 * 4 doubles) receives the average duration in milliseconds of the plan
 * kernel, the sweep kernel(s), the finishing kernels (reduction of the
 * partial sums and, for a refining mixed sweep, the flagging, FP64 refine
 * sweep and scatter) and the whole call.  Outputs as hermite_force_jerk.
 * EINVAL for reps < 1 or a bad size; EHIP when an event call fails. */
int hermite_force_jerk_timed(hermite_ctx* ctx, const hermite_state* s,
                             const hermite_clusters* cl, const int32_t* idx,
                             int32_t n_act, double eps2, int precision,
                             double* acc, double* jerk, double* pot,
                             int32_t reps, double* ms_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * sweep of hermite_force_jerk without a context and without any
 * allocation.  Same arguments and results as hermite_force_jerk with a
 * fresh context's launch shape and mixed-precision policy, except that the
 * device counters are not updated.  Its scratch (plan, cluster tables,
 * partial sums, refinement lists) is one static device array of
 * HERMITE_NOALLOC_SCRATCH_BYTES (about 35 MB) that each GPU the library
 * runs on holds until the process ends; it limits a call to
 * HERMITE_NOALLOC_MAX_ACTIVE active particles and
 * HERMITE_NOALLOC_MAX_CLUSTERS clusters (EINVAL beyond).  The array's
 * device address is looked up once per device, by hermite_create or else
 * by the first call on that device.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race and give wrong results.  Nothing in it needs clearing between
 * calls. */
#define HERMITE_NOALLOC_MAX_ACTIVE   65536
#define HERMITE_NOALLOC_MAX_CLUSTERS 1024
#define HERMITE_NOALLOC_SCRATCH_BYTES 34705932
int hermite_force_jerk_noalloc(const hermite_state* s, const hermite_clusters* cl,
                               const int32_t* idx, const int32_t* n_act_dev,
                               int32_t n_act_max, double eps2, int precision,
                               double* acc, double* jerk, double* pot, void* stream);

/* Procedure steps 5-8 with the snap/crackle, corrector and timestep
 * equations of Section 2: for each active i (idx, n_act as above, T as
 * in hermite_predict), from s->xp, s->vp, the old s->a, s->j and the new
 * compact acc, jerk, pot: corrects s->x, s->v, sets s->a, s->j, s->pot,
 * t_i = T and the next dt_i (criterion at the new time with
 * s1 = s0 + c0 dt, c1 = c0).  crit_out (device [n_act_max], may be NULL)
 * receives the criterion before quantisation. */
int hermite_correct(hermite_ctx* ctx, const hermite_state* s,
                    const int32_t* idx, const int32_t* n_act_dev,
                    int32_t n_act_max, const int64_t* T_dev, int64_t T_host,
                    const double* acc, const double* jerk, const double* pot,
                    const hermite_dt_params* p, double* crit_out,
                    void* stream);

/* First step sizes (no snap or crackle yet; the paper gives no start-up
 * rule): dt0 = eta_s |a| / |j|, quantised at T = 0 with no growth limit;
 * sets t_i = 0.  eta_s = p->eta_init if > 0, else eta_f = eta (paper
 * form) or sqrt(eta) (classic form).  |a|/|j| has no guard against a small
 * initial jerk: with eta_s = eta_f the first step can dominate a run's
 * energy error, and eta_init = eta_f / 16 keeps it below the integration
 * error (the 2x growth limit then reaches the steady step in four steps).
 * Reads s->a, s->j. */
int hermite_init_dt(hermite_ctx* ctx, const hermite_state* s,
                    const hermite_dt_params* p, void* stream);

/* t = 0 set-up: a full sweep at the current x, v (copied to xp, vp)
 * gives a0, j0 and pot, then hermite_init_dt. */
int hermite_initialize(hermite_ctx* ctx, const hermite_state* s,
                       const hermite_clusters* cl, double eps2,
                       int precision, const hermite_dt_params* p,
                       void* stream);

/* Energy check (Section 2 after eq. (pot); Section 4): K = 1/2 sum m v^2
 * and W = 1/2 sum m phi, phi from a separate FP64 potential sweep at the
 * positions s->x.  out_dev (device) receives [K, W] per cluster
 * ([C][2]; [2] for a single system).  Deterministic. */
int hermite_energy(hermite_ctx* ctx, const hermite_state* s,
                   const hermite_clusters* cl, double eps2, double* out_dev,
                   void* stream);

/* ---- whole steps, graphs and runs -------------------------------------- */

/* One block step: select -> predict -> force -> correct, with T and n_act
 * kept on the device (context scratch).  The prediction is fused into the
 * sweep (each j as it is staged, each active i as it is loaded) and into
 * the corrector, so a step touches only the particles the sweep reads;
 * s->xp and s->vp are not written.  With use_graph != 0 the stages are
 * captured once into a HIP graph (per state/cluster/precision/parameter
 * set) and replayed.  Steps past T_end do nothing. */
int hermite_step(hermite_ctx* ctx, const hermite_state* s,
                 const hermite_clusters* cl, double eps2, int precision,
                 const hermite_dt_params* p, int64_t T_end, int use_graph,
                 void* stream);

/* Repeat hermite_step until every particle reaches T_end (ticks; must be
 * a multiple of 2^(tick_bits - k_min)), or until max_steps steps have been
 * launched (max_steps <= 0: no limit; the call can then be repeated to
 * continue).  The host reads the device block time once every sync_every
 * steps, and then also checks the state as hermite_check_finite does:
 * a non-finite state ends the call with HERMITE_ENONFINITE.  With
 * use_graph != 0, runs of 8 consecutive steps are captured as one graph
 * (steps past T_end are no-ops), which removes the gap between graph
 * launches that dominates small systems.
 *
 * Block selection in a run (Section 2's block scheme): at the start of the
 * call the particles are ordered by step size (one pass over t and dt,
 * synchronising `stream`).  When every dt_i is a power of two no finer
 * than 2^(tick_bits - k_max), every t_i a multiple of dt_i and no particle
 * is due before the latest t, the next block time is the first multiple of
 * the smallest occupied step after the last block time and the active
 * block is a prefix of that order, so each step selects in O(n_act) (one
 * kernel; for clusters, each cluster keeps its own order and two kernels
 * re-sort and list the clusters' prefixes, with no workgroup waiting on
 * another) instead of scanning t and dt; otherwise, and for one system of
 * n <= 2048 (selected inside the sweep) or more than 2048 clusters, the
 * run selects as hermite_step does.  Both give the same state bit for bit.
 * Should the order ever be inconsistent (a position out of range, which a
 * state left as the scheme produces it cannot give), the call returns
 * HERMITE_EHIP with a message instead of writing out of range, and the
 * state is not to be trusted.
 *
 * steps_out / interactions_out (host, may be NULL) receive the block-step
 * count and the number of pair interactions (sum over steps of
 * sum_i n_c(i)) of this call; done_out (host, may be NULL) is set to 1 when
 * every particle has reached T_end. */
int hermite_run(hermite_ctx* ctx, const hermite_state* s,
                const hermite_clusters* cl, double eps2, int precision,
                const hermite_dt_params* p, int64_t T_end, int use_graph,
                int32_t sync_every, int64_t max_steps, int64_t* steps_out,
                int64_t* interactions_out, int32_t* done_out, void* stream);

/* Checks that every x, v, a, j value of the state is finite (one pass
 * over the state; synchronises `stream`).  Returns HERMITE_ENONFINITE if
 * one is not: with zero softening two coincident particles give an
 * infinite force (reading of the self-term rule for eps = 0). */
int hermite_check_finite(hermite_ctx* ctx, const hermite_state* s, void* stream);

/* Cumulative device counters since creation (synchronises `stream`):
 * out[0] block steps, out[1] interactions, out[2] clamped steps,
 * out[3] block time T and out[4] n_act of the last step that had active
 * particles, out[5] particles whose mixed-precision sums were refined in
 * FP64 (see hermite_set_mixed_policy). */
int hermite_counters(hermite_ctx* ctx, int64_t out[6], void* stream);

/* Histogram of the active-block sizes of every block step since creation
 * (synchronises `stream`): out[b] for b >= 1 counts steps with
 * 2^(b-1) <= n_act < 2^b; out[0] stays 0 (steps past T_end are not
 * counted anywhere). */
int hermite_block_histogram(hermite_ctx* ctx, int64_t out[33], void* stream);

/* ---- launch shape and autotuner ------------------------------------------ */

int hermite_get_tuning(hermite_ctx* ctx, int precision, hermite_tuning* out);

/* Mixed-precision policy of HERMITE_MIXED, HERMITE_MIXED_2F and
 * HERMITE_MIXED_SP (Section 3.2's split of the pair arithmetic).
 *
 * Near field.  With FP32 pair terms, the error of a particle's sum is a
 * random walk of per-term errors of a few u32 weighted by the terms'
 * magnitudes, so it is led by its nearest pairs.  Pairs with
 * |r| < near_factor * N_c^(-1/3) (N_c the size of the particle's system;
 * in standard N-body units about near_factor mean interparticle spacings
 * of a Plummer core) are summed in FP64 from the same FP64 positions,
 * velocities and masses.  With 0 only the self pair and coincident
 * particles take the FP64 path.
 *
 * FP64 systems.  Systems (the state, or clusters) of fewer than
 * fp64_below particles are swept in FP64 altogether: at those sizes the
 * FP64 sweep is as fast as the FP32 one and exact.
 *
 * Refinement.  HERMITE_MIXED and HERMITE_MIXED_2F also estimate each
 * particle's remaining FP32 error from its sums (the squares of the FP32
 * partial sums over runs of 16 or 32 j) and sum a particle again in FP64 when
 * the estimate exceeds 4e-8 of its acceleration or jerk: particles whose
 * sums almost cancel.  The count is reported by hermite_counters.
 *
 * Defaults: near_factor 3, fp64_below 32768 for HERMITE_MIXED and
 * HERMITE_MIXED_2F; 0 and 0 for HERMITE_MIXED_SP (the scheme as printed).
 * EINVAL for HERMITE_FP64, a negative, infinite or NaN near_factor, a
 * negative fp64_below, or fp64_below != 0 for HERMITE_MIXED_SP.  Setting
 * the policy drops captured step graphs. */
int hermite_set_mixed_policy(hermite_ctx* ctx, int precision, double near_factor,
                             int64_t fp64_below);
int hermite_get_mixed_policy(hermite_ctx* ctx, int precision, double* near_factor,
                             int64_t* fp64_below);

/* Small blocks of HERMITE_MIXED and HERMITE_MIXED_2F.  A force sweep (or a
 * block step's sweep) of fewer than fp64_inter_below interactions
 * (sum over systems of active particles x system size) is done in FP64:
 * such a sweep is bound by launch and memory latency, where the FP32
 * arithmetic saves less than the refinement's kernels cost.  Decided on
 * the device from the block's active count, so a captured step adapts to
 * every block.  Default 5e7 (about 760 active particles of a 65536-particle
 * system); 0 sweeps every block with FP32 pair arithmetic.  EINVAL for
 * another precision or a negative value.  Setting it drops captured step
 * graphs. */
int hermite_set_mixed_small_blocks(hermite_ctx* ctx, int precision,
                                   int64_t fp64_inter_below);
int hermite_get_mixed_small_blocks(hermite_ctx* ctx, int precision,
                                   int64_t* fp64_inter_below);
int hermite_set_tuning(hermite_ctx* ctx, int precision,
                       const hermite_tuning* in);

/* Time candidate launch shapes (variant, i.e. particles per lane, FP32
 * difference form and FP32 run length; workgroups per CU, j-split target,
 * minimum j-run) of the sweep for this state (and clusters, may be
 * NULL), precision and active count (the first n_act particles) with HIP
 * events at the predicted positions s->xp, s->vp, and keep the fastest
 * whose results stay as close to an FP64 sweep as the precision allows
 * (FP64: 1e-13 relative; mixed: 1e-6 or 1.5 times the default shape's
 * deviation, whichever is larger).  Every candidate is screened with a few
 * launches; the six fastest and the default are then timed again in three
 * interleaved rounds, and the lowest median wins.  Installs it in the
 * context and, if cache_path is non-NULL, merges it into that JSON file
 * keyed by device architecture, HIP version, precision and power-of-two
 * size buckets of n and n_act, with its time and the HBM bytes its j-split
 * adds (partial sums written and read back).  Synchronises. */
int hermite_autotune(hermite_ctx* ctx, const hermite_state* s,
                     const hermite_clusters* cl, double eps2, int precision,
                     int32_t n_act, const char* cache_path, void* stream);

/* Load tunings from a cache written by hermite_autotune for this device
 * and the given n / n_act bucket; returns HERMITE_OK if an entry was
 * found and installed, HERMITE_EINVAL if none matched. */
int hermite_load_tuning(hermite_ctx* ctx, const char* cache_path,
                        int precision, int64_t n, int32_t n_act);

#ifdef __cplusplus
}
#endif

#endif /* HERMITE_H */
