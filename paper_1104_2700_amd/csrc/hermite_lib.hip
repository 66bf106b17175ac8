// Host side of libhermite: the C ABI of include/hermite.h, argument
// validation, context scratch, HIP graph capture/replay and the autotuner.
#include "hermite.h"
#include "hermite_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

using namespace hm;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            return fail(HERMITE_EHIP, "%s: %s (%s:%d)", #call,                \
                        hipGetErrorString(e_), __FILE__, __LINE__);           \
    } while (0)

#define CHECK(code)                                                           \
    do {                                                                      \
        int c_ = (code);                                                      \
        if (c_ != HERMITE_OK) return c_;                                      \
    } while (0)

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Block steps per graph in hermite_run: one graph launch costs about as
// much as a small system's whole step, so runs replay several steps each.
constexpr int kRunGraphSteps = 8;

struct GraphEntry {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct hermite_ctx {
    int device = 0;
    int n_cu = 0;
    std::string arch;
    hipStream_t cap_stream = nullptr;
    hermite_tuning tuning[4];
    double near_factor[4];     // near-field radius factor per precision
    int64_t fp64_below[4];     // systems smaller than this are swept in FP64
    int64_t fp64_inter_below[4];   // blocks of fewer interactions are swept in FP64
    // scratch
    Buf plan, act_start, act_cnt, chunks, item_off, partial;
    // refinement of mixed sweeps: flags and lists, the refine sweep's plan,
    // per-cluster tables and partial sums, and the flagging reduce's ticket
    Buf ref_pos, ref_idx, ref_p, ref_tmp, ref_ucnt, ref_ccnt, rplan, ract_start, ract_cnt,
        rchunks, ritem_off;
    Buf sel_min, sel_cnt;
    Buf step_idx, step_na, step_T, step_out, step_acl, phi, counters, ticket, flag;
    // step-size order of a run (hermite_run)
    Buf lvl_perm, lvl_tmp, lvl_cnt, lvl_cursor, lvl_misc, lvl_na, lvl_bits, lvl_lv, lvl_cst;
    Buf lvl_ccnt, lvl_ccum, lvl_cna;   // ensembles: per-cluster orders
    std::vector<GraphEntry> graphs;
    // grid of the fused select + sweep for the last shape it was sized for
    struct {
        int64_t n = -1, cap = 0;
        int32_t lanes = 0, min_j = 0, ipl = 0, grid = 0;
    } fused;
};

namespace {

void drop_graphs(hermite_ctx* c)
{
    for (auto& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// Grow a scratch buffer; every growth invalidates captured graphs.
int ensure(hermite_ctx* c, Buf& b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return HERMITE_OK;
    drop_graphs(c);
    if (b.p) {
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(HERMITE_ENOMEM, "scratch allocation of %zu bytes failed", bytes);
    }
    b.p = p;
    b.bytes = bytes;
    return HERMITE_OK;
}

int check_ctx(hermite_ctx* c)
{
    if (!c) return fail(HERMITE_EINVAL, "null context");
    HIP_OK(hipSetDevice(c->device));
    return HERMITE_OK;
}

int check_state(const hermite_state* s)
{
    if (!s) return fail(HERMITE_EINVAL, "null state");
    if (s->n < 1 || s->n > INT32_MAX)
        return fail(HERMITE_EINVAL, "n = %lld out of range [1, 2^31-1]", (long long)s->n);
    if (s->tick_bits < 1 || s->tick_bits > 52)
        return fail(HERMITE_EINVAL, "tick_bits = %d out of range [1, 52]", s->tick_bits);
    if (!s->m || !s->x || !s->v || !s->a || !s->j || !s->xp || !s->vp || !s->pot || !s->t || !s->dt)
        return fail(HERMITE_EINVAL, "null pointer in hermite_state");
    return HERMITE_OK;
}

int check_precision(int precision)
{
    if (precision < HERMITE_FP64 || precision > HERMITE_MIXED_SP)
        return fail(HERMITE_EINVAL, "unknown precision %d", precision);
    return HERMITE_OK;
}

int check_eps2(double eps2)
{
    if (!(eps2 >= 0.0) || std::isinf(eps2))
        return fail(HERMITE_EINVAL, "eps2 must be finite and >= 0");
    return HERMITE_OK;
}

int check_clusters(const hermite_clusters* cl, int64_t n)
{
    if (!cl) return HERMITE_OK;
    if (cl->n_clusters < 1) return fail(HERMITE_EINVAL, "n_clusters must be >= 1");
    if (!cl->offsets || !cl->eps2) return fail(HERMITE_EINVAL, "null cluster arrays");
    if (cl->max_size < 1 || cl->max_size > n)
        return fail(HERMITE_EINVAL, "cluster max_size %lld out of range [1, n]",
                    (long long)cl->max_size);
    return HERMITE_OK;
}

int check_dt(const hermite_dt_params* p, int tick_bits)
{
    if (!p) return fail(HERMITE_EINVAL, "null dt params");
    if (!(p->eta > 0.0) || std::isinf(p->eta)) return fail(HERMITE_EINVAL, "eta must be > 0");
    if (!(p->eta_init >= 0.0) || std::isinf(p->eta_init))
        return fail(HERMITE_EINVAL, "eta_init must be >= 0 (0 = default)");
    if (p->form != HERMITE_DT_PAPER && p->form != HERMITE_DT_AARSETH)
        return fail(HERMITE_EINVAL, "unknown timestep form %d", p->form);
    if (p->k_min < 0 || p->k_max < p->k_min || p->k_max > tick_bits)
        return fail(HERMITE_EINVAL, "need 0 <= k_min <= k_max <= tick_bits (%d, %d, %d)",
                    p->k_min, p->k_max, tick_bits);
    return HERMITE_OK;
}

// Default launch shape: two active particles per lane (variant 1), five
// persistent workgroups per CU, and a work split aiming at one item per
// workgroup of the grid.
// Chosen from a sweep of these parameters over active counts 256 ... 65536
// at N = 65536 on gfx950; hermite_autotune refines it per size.
hermite_tuning default_tuning_for(int n_cu)
{
    hermite_tuning t;
    t.variant = 1;
    t.wg_per_cu = 5;
    t.target_lanes = n_cu * t.wg_per_cu * kWG;
    t.min_j_per_lane = 4;
    return t;
}

hermite_tuning default_tuning(const hermite_ctx* c, int precision)
{
    (void)precision;
    return default_tuning_for(c->n_cu);
}

// Mixed-precision policy (hermite_set_mixed_policy).  Near-field radius
// factor, in N_c^(-1/3) (about one mean interparticle spacing of a Plummer
// core in standard units): the FP32 pair error of a particle is led by its
// nearest pairs, whose terms are the largest, so HERMITE_MIXED and
// HERMITE_MIXED_2F sum the pairs within this radius in FP64.  Systems
// smaller than fp64_below are swept in FP64 altogether: up to about 2^15
// particles the FP64 sweep of all of them takes no longer than the FP32 one
// with its near field and refinement (MI355X, default launch shapes: FP64 /
// mixed 0.019 / 0.042 ms at N = 1024, 0.044 / 0.074 at 4096, 0.364 / 0.354
// at 16384; 5.07 / 4.04 at 65536), and whole runs take the mixed path's
// extra launches on every block step (N = 16384, t = 0 -> 1: 6.7 s against
// 5.2 s in FP64).  The paper-faithful
// mode keeps the printed scheme: radius 0 (only the self pair and
// coincident particles take the FP64 path) and no FP64 systems.
double default_near_factor(int precision)
{
    return (precision == HERMITE_MIXED || precision == HERMITE_MIXED_2F) ? 3.0 : 0.0;
}

int64_t default_fp64_below(int precision)
{
    return (precision == HERMITE_MIXED || precision == HERMITE_MIXED_2F) ? 32768 : 0;
}

// Blocks of fewer interactions than this are swept in FP64 by the mixed
// precisions: a small block's sweep is bound by launch and load latency,
// and the refinement's extra launches cost more than FP32 arithmetic saves
// (MI355X, N = 65536, autotuned shapes: FP64 / mixed 57 / 71 us at 512
// active particles, 100 / 103 at 1024, 183 / 176 at 2048).
int64_t default_fp64_inter_below(int precision)
{
    return (precision == HERMITE_MIXED || precision == HERMITE_MIXED_2F) ? 50000000 : 0;
}

// Device scratch of one force sweep and of its refinement, as pointers
// (context buffers, or the static scratch of hermite_force_jerk_noalloc).
struct SweepScratch {
    SweepPlan* plan;
    int32_t *act_start, *act_cnt, *chunks, *item_off;   // [C], item_off [C+1]
    double* partial;
    int64_t partial_cap;                                // doubles
    int32_t *ref_pos, *ref_idx, *ref_p, *ref_tmp;       // [n_act_max]
    int32_t *ref_ucnt, *ref_ccnt;                       // [n_act_max / 4 + 1], [C]
    SweepPlan* rplan;
    int32_t *ract_start, *ract_cnt, *rchunks, *ritem_off;
};

// Partial-sum capacity of a sweep (doubles) for an active count: room for
// 32 j-chunks of every active particle.  The refine sweep reuses the same
// buffer: its partials are written after the flagging reduce has read the
// sweep's.
int64_t partial_cap_for(int32_t n_act_max)
{
    return (int64_t)kRows * 32 * std::max<int64_t>(n_act_max, 4096);
}

// True when a sweep of this precision and these systems runs the FP64
// refinement: the mixed precisions, when some system is swept in FP32.
bool uses_refine(int precision, int64_t n_cmax, int64_t fp64_below)
{
    return (precision == HERMITE_MIXED || precision == HERMITE_MIXED_2F) && n_cmax >= fp64_below;
}

// Fills the sweep arguments from a state, launch shape, mixed policy and
// scratch (no allocation).
void fill_sweep(const SweepScratch& sc, const hermite_state* s, const hermite_clusters* cl,
                const double* xp, const double* vp, const int32_t* idx,
                const int32_t* n_act_dev, int32_t n_act_max, double eps2, int precision,
                const hermite_tuning& tu, double near_factor, int64_t fp64_below,
                int64_t fp64_inter_below, int64_t* counters, double* acc, double* jerk,
                double* pot, SweepArgs* a)
{
    std::memset(a, 0, sizeof *a);
    a->xp = xp;
    a->vp = vp;
    a->m = s->m;
    a->n = s->n;
    a->idx = idx;
    a->n_act_dev = n_act_dev;
    a->n_act_max = n_act_max;
    a->n_clusters = cl ? cl->n_clusters : 1;
    a->offsets = cl ? cl->offsets : nullptr;
    a->eps2_c = cl ? cl->eps2 : nullptr;
    a->eps2 = eps2;
    a->n_cmax = cl ? cl->max_size : s->n;
    a->plan = sc.plan;
    a->act_start = sc.act_start;
    a->act_cnt = sc.act_cnt;
    a->chunks = sc.chunks;
    a->item_off = sc.item_off;
    a->partial = sc.partial;
    a->partial_cap = sc.partial_cap;
    a->target_lanes = tu.target_lanes;
    a->min_j_per_lane = tu.min_j_per_lane;
    a->near_factor = precision == HERMITE_FP64 ? 0.0 : near_factor;
    a->fp64_below = precision == HERMITE_FP64 ? 0 : fp64_below;
    a->fp64_inter_below =
        (precision == HERMITE_MIXED || precision == HERMITE_MIXED_2F) ? fp64_inter_below : 0;
    a->refine = uses_refine(precision, a->n_cmax, a->fp64_below) ? 1 : 0;
    if (a->refine) {
        a->ref_pos = sc.ref_pos;
        a->ref_idx = sc.ref_idx;
        a->ref_p = sc.ref_p;
        a->ref_tmp = sc.ref_tmp;
        a->ref_ucnt = sc.ref_ucnt;
        a->ref_ccnt = sc.ref_ccnt;
    }
    a->one_chunk = precision == HERMITE_MIXED_SP ? 1 : 0;
    a->counters = counters;
    a->acc = acc;
    a->jerk = jerk;
    a->pot = pot;
}

// The FP64 refine sweep of a mixed sweep with refinement: the same system
// and prediction, the flagged particles (ref_idx) as its active list, and
// scratch of its own (its plan is made on the device after the flagging
// reduce).
void fill_refine(const SweepScratch& sc, const SweepArgs& a, SweepArgs* ra)
{
    *ra = a;
    ra->idx = a.ref_idx;
    ra->n_act_dev = nullptr;
    ra->plan = sc.rplan;
    ra->act_start = sc.ract_start;
    ra->act_cnt = sc.ract_cnt;
    ra->chunks = sc.rchunks;
    ra->item_off = sc.ritem_off;
    ra->act_cluster = nullptr;
    // with clusters the refine list's builder writes each cluster's run start
    ra->sel_clusters = a.n_clusters > 1 ? 1 : 0;
    // the sweep's partial sums are consumed (by the flagging reduce) before
    // the refine sweep writes its own, so both use one buffer; an FP64 block
    // then gets the sweep's own split
    ra->partial = sc.partial;
    ra->partial_cap = sc.partial_cap;
    ra->refine = 0;
    ra->defer_fp64 = 0;
    ra->near_factor = 0.0;
    ra->fp64_below = 0;
    ra->fp64_inter_below = 0;
    ra->kind = 0;
    ra->counters = nullptr;
    ra->sel_dt = nullptr;
    ra->sel_idx_out = nullptr;
    ra->sel_na_out = nullptr;
    ra->sel_T_out = nullptr;
    ra->acc = ra->jerk = ra->pot = nullptr;
}

// The context's scratch for a sweep of C systems and n_act_max active
// particles (allocated or grown as needed).
int ctx_scratch(hermite_ctx* c, int C, int32_t n_act_max, bool refine, SweepScratch* sc)
{
    std::memset(sc, 0, sizeof *sc);
    CHECK(ensure(c, c->plan, sizeof(SweepPlan)));
    CHECK(ensure(c, c->act_start, sizeof(int32_t) * C));
    CHECK(ensure(c, c->act_cnt, sizeof(int32_t) * C));
    CHECK(ensure(c, c->chunks, sizeof(int32_t) * C));
    CHECK(ensure(c, c->item_off, sizeof(int32_t) * (C + 1)));
    CHECK(ensure(c, c->partial, sizeof(double) * partial_cap_for(n_act_max)));
    sc->plan = (SweepPlan*)c->plan.p;
    sc->act_start = (int32_t*)c->act_start.p;
    sc->act_cnt = (int32_t*)c->act_cnt.p;
    sc->chunks = (int32_t*)c->chunks.p;
    sc->item_off = (int32_t*)c->item_off.p;
    sc->partial = (double*)c->partial.p;
    sc->partial_cap = (int64_t)(c->partial.bytes / sizeof(double));
    if (refine) {
        const size_t na = (size_t)std::max<int32_t>(n_act_max, 1);
        CHECK(ensure(c, c->ref_pos, sizeof(int32_t) * na));
        CHECK(ensure(c, c->ref_idx, sizeof(int32_t) * na));
        CHECK(ensure(c, c->ref_p, sizeof(int32_t) * na));
        CHECK(ensure(c, c->ref_tmp, sizeof(int32_t) * na));
        CHECK(ensure(c, c->ref_ucnt, sizeof(int32_t) * (na / (kWG / 64) + 1)));
        CHECK(ensure(c, c->ref_ccnt, sizeof(int32_t) * (size_t)C));
        CHECK(ensure(c, c->rplan, sizeof(SweepPlan)));
        CHECK(ensure(c, c->ract_start, sizeof(int32_t) * C));
        CHECK(ensure(c, c->ract_cnt, sizeof(int32_t) * C));
        CHECK(ensure(c, c->rchunks, sizeof(int32_t) * C));
        CHECK(ensure(c, c->ritem_off, sizeof(int32_t) * (C + 1)));
        sc->ref_pos = (int32_t*)c->ref_pos.p;
        sc->ref_idx = (int32_t*)c->ref_idx.p;
        sc->ref_p = (int32_t*)c->ref_p.p;
        sc->ref_tmp = (int32_t*)c->ref_tmp.p;
        sc->ref_ucnt = (int32_t*)c->ref_ucnt.p;
        sc->ref_ccnt = (int32_t*)c->ref_ccnt.p;
        sc->rplan = (SweepPlan*)c->rplan.p;
        sc->ract_start = (int32_t*)c->ract_start.p;
        sc->ract_cnt = (int32_t*)c->ract_cnt.p;
        sc->rchunks = (int32_t*)c->rchunks.p;
        sc->ritem_off = (int32_t*)c->ritem_off.p;
    }
    return HERMITE_OK;
}

// Fills the sweep arguments and makes sure the context scratch they point
// to exists (refinement scratch included, when the sweep refines).
int prepare_sweep(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                  const double* xp, const double* vp, const int32_t* idx,
                  const int32_t* n_act_dev, int32_t n_act_max, double eps2, int precision,
                  const hermite_tuning& tu, double* acc, double* jerk, double* pot,
                  SweepArgs* a)
{
    const int C = cl ? cl->n_clusters : 1;
    const double nfac = precision == HERMITE_FP64 ? 0.0 : c->near_factor[precision];
    const int64_t f64b = precision == HERMITE_FP64 ? 0 : c->fp64_below[precision];
    const bool refine = uses_refine(precision, cl ? cl->max_size : s->n, f64b);
    SweepScratch sc;
    CHECK(ctx_scratch(c, C, n_act_max, refine, &sc));
    CHECK(ensure(c, c->counters, sizeof(int64_t) * kCounters));
    fill_sweep(sc, s, cl, xp, vp, idx, n_act_dev, n_act_max, eps2, precision, tu, nfac, f64b,
               c->fp64_inter_below[precision], (int64_t*)c->counters.p, acc, jerk, pot, a);
    return HERMITE_OK;
}

// The refine sweep's arguments from the context scratch (which
// prepare_sweep has made for a refining sweep).
int prepare_refine(hermite_ctx* c, const SweepArgs& a, SweepArgs* ra)
{
    SweepScratch sc;
    CHECK(ctx_scratch(c, a.n_clusters, a.n_act_max, true, &sc));
    fill_refine(sc, a, ra);
    return HERMITE_OK;
}

int run_force(hermite_ctx* c, const SweepArgs& a, int precision, const hermite_tuning& tu,
              bool pot_only, hipStream_t st)
{
    const int grid = std::max(1, c->n_cu * tu.wg_per_cu);
    SweepArgs ra;
    if (a.refine && !pot_only) CHECK(prepare_refine(c, a, &ra));
    HIP_OK(launch_force(a, (a.refine && !pot_only) ? &ra : nullptr, precision, tu.variant, grid,
                        pot_only, st));
    return HERMITE_OK;
}

int ensure_step_scratch(hermite_ctx* c, int64_t n)
{
    CHECK(ensure(c, c->step_idx, sizeof(int32_t) * n));
    CHECK(ensure(c, c->step_acl, sizeof(int32_t) * n));
    CHECK(ensure(c, c->step_na, sizeof(int32_t) * 2));
    CHECK(ensure(c, c->step_T, sizeof(int64_t) * 2));
    CHECK(ensure(c, c->step_out, sizeof(double) * 7 * n));
    const int nb = select_blocks(n);
    CHECK(ensure(c, c->sel_min, sizeof(int64_t) * nb));
    CHECK(ensure(c, c->sel_cnt, sizeof(int32_t) * nb));
    CHECK(ensure(c, c->counters, sizeof(int64_t) * kCounters));
    if (!c->ticket.p) {
        CHECK(ensure(c, c->ticket, sizeof(uint32_t) * 4));
        HIP_OK(hipMemset(c->ticket.p, 0, sizeof(uint32_t) * 4));
    }
    return HERMITE_OK;
}

LevelArgs level_args(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                     const hermite_dt_params* p, int64_t T_end)
{
    LevelArgs L;
    std::memset(&L, 0, sizeof L);
    L.n = s->n;
    L.t = s->t;
    L.dt = s->dt;
    L.dt_floor = ((int64_t)1) << (s->tick_bits - p->k_max);
    L.perm = (int32_t*)c->lvl_perm.p;
    L.cnt = (int32_t*)c->lvl_cnt.p;
    L.cursor = (int32_t*)c->lvl_cursor.p;
    L.misc = (int64_t*)c->lvl_misc.p;
    L.tmp = (int32_t*)c->lvl_tmp.p;
    L.na_prev = (int32_t*)c->lvl_na.p;
    L.bits = (uint32_t*)c->lvl_bits.p;
    L.T_end = T_end;
    L.na = (int32_t*)c->step_na.p;
    L.T = (int64_t*)c->step_T.p;
    L.idx = (int32_t*)c->step_idx.p;
    L.lv = (const uint8_t*)c->lvl_lv.p;
    L.counters = (int64_t*)c->counters.p;
    L.n_clusters = cl ? cl->n_clusters : 1;
    if (cl && cl->n_clusters > 1) {
        L.offsets = cl->offsets;
        L.ccnt = (int32_t*)c->lvl_ccnt.p;
        L.ccum = (int32_t*)c->lvl_ccum.p;
        L.cna = (int32_t*)c->lvl_cna.p;
        L.cst = (int32_t*)c->lvl_cst.p;
    }
    return L;
}

// Builds the step-size order of s for a run (per cluster for ensembles;
// synchronises st).  *ok is false when the state is not one the block
// scheme can have produced (the run then selects every block from t and
// dt).
int level_init(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
               const hermite_dt_params* p, hipStream_t st, bool* ok)
{
    *ok = false;
    CHECK(ensure(c, c->lvl_perm, sizeof(int32_t) * s->n));
    CHECK(ensure(c, c->lvl_tmp, sizeof(int32_t) * s->n));
    CHECK(ensure(c, c->lvl_cnt, sizeof(int32_t) * 64));
    CHECK(ensure(c, c->lvl_cursor, sizeof(int32_t) * 64));
    CHECK(ensure(c, c->lvl_misc, sizeof(int64_t) * 8));
    CHECK(ensure(c, c->lvl_na, sizeof(int32_t) * 2));
    CHECK(ensure(c, c->lvl_bits, sizeof(uint32_t) * ((s->n + 31) / 32)));
    CHECK(ensure(c, c->lvl_lv, sizeof(uint8_t) * s->n));
    if (cl && cl->n_clusters > 1) {
        const size_t C = (size_t)cl->n_clusters;
        CHECK(ensure(c, c->lvl_ccnt, sizeof(int32_t) * 64 * C));
        CHECK(ensure(c, c->lvl_ccum, sizeof(int32_t) * 64 * C));
        CHECK(ensure(c, c->lvl_cna, sizeof(int32_t) * C));
        CHECK(ensure(c, c->lvl_cst, sizeof(int32_t) * C));
    }
    const LevelArgs L = level_args(c, s, cl, p, 0);
    const int64_t init[8] = {0, INT64_MIN, INT64_MAX, 0, 0, 0, 0, 0};
    HIP_OK(hipMemcpyAsync(L.misc, init, sizeof init, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(L.cnt, 0, sizeof(int32_t) * 64, st));
    HIP_OK(hipMemsetAsync(L.cursor, 0, sizeof(int32_t) * 64, st));
    HIP_OK(hipMemsetAsync(L.na_prev, 0, sizeof(int32_t) * 2, st));
    HIP_OK(hipMemsetAsync(L.bits, 0, sizeof(uint32_t) * ((s->n + 31) / 32), st));
    // every entry of the active list and its clusters holds a valid index
    // from the start, whatever a step writes
    HIP_OK(hipMemsetAsync(c->step_idx.p, 0, sizeof(int32_t) * s->n, st));
    HIP_OK(hipMemsetAsync(c->step_acl.p, 0, sizeof(int32_t) * s->n, st));
    HIP_OK(launch_level_count(L, st));
    int64_t h[4];
    HIP_OK(hipMemcpyAsync(h, L.misc, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (h[3] != 0 || h[1] >= h[2]) return HERMITE_OK;
    HIP_OK(launch_level_build(L, st));
    *ok = true;
    return HERMITE_OK;
}

// One block step on stream st using the context's step scratch: selection
// with the sweep plan (from the step-size order in a run, one kernel;
// otherwise from t and dt: two kernels, one up to 4096 particles, or
// inside the sweep for one system of up to kFusedSelMax), the persistent
// sweep (predicting the particles it reads), and the fused reduce +
// correct.
int enqueue_step(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                 double eps2, int precision, const hermite_dt_params* p, int64_t T_end,
                 bool level, hipStream_t st)
{
    const int64_t n = s->n;
    int32_t* idx = (int32_t*)c->step_idx.p;
    int32_t* na = (int32_t*)c->step_na.p;
    int64_t* T = (int64_t*)c->step_T.p;
    double* out = (double*)c->step_out.p;
    int64_t* counters = (int64_t*)c->counters.p;
    // one system in a run: the active block is the prefix of the order
    int32_t* aidx = (level && !cl) ? (int32_t*)c->lvl_perm.p : idx;
    SweepArgs a;
    const hermite_tuning& tu = c->tuning[precision];
    CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, aidx, na, (int32_t)n, eps2, precision, tu, out,
                        out + 3 * n, out + 6 * n, &a));
    a.ipl = (tu.variant & 1) ? 2 : 1;
    // a block the plan puts in FP64 takes the refine sweep's launch (over
    // the whole block) and the corrector's reduce
    a.defer_fp64 = a.refine;
    // with clusters the selection records the active runs and clusters
    a.act_cluster = cl ? (int32_t*)c->step_acl.p : nullptr;
    a.sel_clusters = cl ? 1 : 0;
    // prediction happens inside the sweep and the corrector (no pass over
    // the whole state: only particles a sweep touches are predicted)
    a.pred_x = s->x;
    a.pred_v = s->v;
    a.pred_a = s->a;
    a.pred_j = s->j;
    a.pred_t = s->t;
    a.pred_T = T;
    a.tick = std::ldexp(1.0, -s->tick_bits);
    const int grid = std::max(1, c->n_cu * tu.wg_per_cu);
    if (level) {
        HIP_OK(launch_level_select(level_args(c, s, cl, p, T_end), a, st));
        HIP_OK(launch_sweep_only(a, precision, tu.variant, grid, st));
    } else if (!cl && n <= kFusedSelMax) {
        // one small system: every sweep workgroup selects the block itself
        // (no selection kernel); the grid is capped at the most items any
        // active count can give, so idle workgroups do no selection
        a.sel_dt = s->dt;
        a.sel_T_end = T_end;
        a.sel_idx_out = idx;
        a.sel_na_out = na;
        a.sel_T_out = T;
        auto& f = c->fused;
        if (f.n != n || f.cap != a.partial_cap || f.lanes != a.target_lanes ||
            f.min_j != a.min_j_per_lane || f.ipl != a.ipl) {
            f.n = n;
            f.cap = a.partial_cap;
            f.lanes = a.target_lanes;
            f.min_j = a.min_j_per_lane;
            f.ipl = a.ipl;
            f.grid = max_plan_items(a);
        }
        HIP_OK(launch_select_sweep(a, precision, tu.variant, std::min(grid, f.grid), st));
    } else {
        HIP_OK(launch_step_select(n, s->t, s->dt, T_end, idx, na, T, (int64_t*)c->sel_min.p,
                                  (int32_t*)c->sel_cnt.p, counters, (uint32_t*)c->ticket.p, a,
                                  st));
        HIP_OK(launch_sweep_only(a, precision, tu.variant, grid, st));
    }
    CorrectArgs ca;
    std::memset(&ca, 0, sizeof ca);
    ca.n = n;
    ca.tick_bits = s->tick_bits;
    ca.idx = aidx;
    ca.n_act_dev = na;
    ca.n_act_max = (int32_t)n;
    ca.T_dev = T;
    ca.xp = s->xp;
    ca.vp = s->vp;
    ca.x = s->x;
    ca.v = s->v;
    ca.a = s->a;
    ca.j = s->j;
    ca.pot = s->pot;
    ca.t = s->t;
    ca.dt = s->dt;
    ca.eta = p->eta;
    ca.form = p->form;
    ca.k_min = p->k_min;
    ca.k_max = p->k_max;
    ca.counters = counters;
    ca.predict_i = 1;
    if (level) {
        ca.na_seen = (int32_t*)c->lvl_na.p;
        ca.lv_out = (uint8_t*)c->lvl_lv.p;
    }
    if (a.refine) {
        // mixed sums into the compact outputs with their error flags, the
        // FP64 refine sweep of the flagged particles, then the corrector
        SweepArgs ra;
        CHECK(prepare_refine(c, a, &ra));
        HIP_OK(launch_reduce_refine(a, ra, tu.variant, grid, st));
        ca.acc1 = out;
        ca.jrk1 = out + 3 * n;
        ca.pot1 = out + 6 * n;
        HIP_OK(launch_correct_refine(ca, a, ra, st));
    } else {
        HIP_OK(launch_correct_reduce(ca, a, st));
    }
    return HERMITE_OK;
}

std::string step_key(const hermite_state* s, const hermite_clusters* cl, double eps2,
                     int precision, const hermite_dt_params* p, int64_t T_end,
                     const hermite_tuning& tu)
{
    std::ostringstream k;
    k << s->n << '|' << s->tick_bits << '|' << (const void*)s->m << (void*)s->x
      << (void*)s->v << (void*)s->a << (void*)s->j << (void*)s->xp << (void*)s->vp
      << (void*)s->pot << (void*)s->t << (void*)s->dt << '|';
    if (cl)
        k << cl->n_clusters << ',' << cl->max_size << ',' << (const void*)cl->offsets
          << (const void*)cl->eps2;
    uint64_t eb;
    std::memcpy(&eb, &eps2, 8);
    uint64_t etab;
    std::memcpy(&etab, &p->eta, 8);
    k << '|' << eb << '|' << precision << '|' << etab << ',' << p->form << ','
      << p->k_min << ',' << p->k_max << '|' << T_end << '|' << tu.target_lanes << ','
      << tu.wg_per_cu << ',' << tu.min_j_per_lane << ',' << tu.variant;
    return k.str();
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of hermite_force_jerk_noalloc: one file-scope device array, laid
// out as the context scratch of a sweep of at most kNoAllocMaxActive active
// particles in at most kNoAllocMaxClusters systems (partial sums for 8
// j-chunks of every active particle, shared with the refine sweep).  Each device
// holds its own copy, at the address hipGetSymbolAddress gives on it.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxActive = HERMITE_NOALLOC_MAX_ACTIVE;
constexpr int kNoAllocMaxClusters = HERMITE_NOALLOC_MAX_CLUSTERS;
constexpr int64_t kNoAllocPartial = (int64_t)kRows * 8 * kNoAllocMaxActive;    // doubles
constexpr int64_t kNoAllocInts =
    2 * (3 * (int64_t)kNoAllocMaxClusters + (kNoAllocMaxClusters + 1)) +  // tables
    4 * kNoAllocMaxActive + (kNoAllocMaxActive / (kWG / 64) + 1) +         // refine lists
    kNoAllocMaxClusters;                                                    // per-cluster counts
constexpr size_t kNoAllocBytes = sizeof(double) * kNoAllocPartial +
                                 2 * 256 +                                  // the two plans
                                 sizeof(int32_t) * kNoAllocInts;
static_assert(sizeof(SweepPlan) <= 256, "plan slot");
static_assert(kNoAllocBytes == (size_t)HERMITE_NOALLOC_SCRATCH_BYTES, "header states the size");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

struct NoAllocDevice {
    bool ready = false;
    unsigned char* base = nullptr;   // the array's address on this device
    int n_cu = 0;
};

std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[64];

// Once per device, with it current: the array's address there (host code
// must never pass the array's own name, a host-side stand-in) and the CU
// count for the launch shape.
int noalloc_init(int device, NoAllocDevice** out)
{
    if (device < 0 || device >= 64) return fail(HERMITE_ENODEV, "device %d not supported", device);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocDevice& d = g_noalloc[device];
    if (!d.ready) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        int n_cu = 0;
        HIP_OK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
        d.base = (unsigned char*)ptr;
        d.n_cu = n_cu;
        d.ready = true;
    }
    *out = &d;
    return HERMITE_OK;
}

// The SweepScratch views of the static array on one device.
SweepScratch noalloc_carve(unsigned char* base)
{
    SweepScratch sc;
    std::memset(&sc, 0, sizeof sc);
    double* d = (double*)base;
    sc.partial = d;
    sc.partial_cap = kNoAllocPartial;
    unsigned char* q = (unsigned char*)(d + kNoAllocPartial);
    sc.plan = (SweepPlan*)q;
    sc.rplan = (SweepPlan*)(q + 256);
    int32_t* i = (int32_t*)(q + 512);
    const int C = kNoAllocMaxClusters;
    sc.act_start = i;   i += C;
    sc.act_cnt = i;     i += C;
    sc.chunks = i;      i += C;
    sc.item_off = i;    i += C + 1;
    sc.ract_start = i;  i += C;
    sc.ract_cnt = i;    i += C;
    sc.rchunks = i;     i += C;
    sc.ritem_off = i;   i += C + 1;
    sc.ref_pos = i;     i += kNoAllocMaxActive;
    sc.ref_idx = i;     i += kNoAllocMaxActive;
    sc.ref_p = i;       i += kNoAllocMaxActive;
    sc.ref_tmp = i;     i += kNoAllocMaxActive;
    sc.ref_ucnt = i;    i += kNoAllocMaxActive / (kWG / 64) + 1;
    sc.ref_ccnt = i;
    return sc;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* hermite_last_error(void) { return g_err.c_str(); }

int hermite_create(int device, hermite_ctx** out)
{
    if (!out) return fail(HERMITE_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return fail(HERMITE_ENODEV, "no HIP device available");
    }
    if (device < 0 || device >= count)
        return fail(HERMITE_ENODEV, "device %d not in [0, %d)", device, count);
    HIP_OK(hipSetDevice(device));
    hermite_ctx* c = new hermite_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return fail(HERMITE_EHIP, "hipGetDeviceProperties failed");
    }
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    {
        // set-up of hermite_force_jerk_noalloc's scratch on this device
        NoAllocDevice* nd = nullptr;
        const int rc0 = noalloc_init(device, &nd);
        if (rc0 != HERMITE_OK) {
            delete c;
            return rc0;
        }
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(HERMITE_EHIP, "hipStreamCreateWithFlags failed");
    }
    for (int p = 0; p < 4; ++p) {
        c->tuning[p] = default_tuning(c, p);
        c->near_factor[p] = default_near_factor(p);
        c->fp64_below[p] = default_fp64_below(p);
        c->fp64_inter_below[p] = default_fp64_inter_below(p);
    }
    int rc = ensure(c, c->counters, sizeof(int64_t) * kCounters);
    if (rc == HERMITE_OK && hipMemset(c->counters.p, 0, sizeof(int64_t) * kCounters) != hipSuccess)
        rc = fail(HERMITE_EHIP, "hipMemset of counters failed");
    if (rc != HERMITE_OK) {
        hermite_destroy(c);
        return rc;
    }
    *out = c;
    return HERMITE_OK;
}

int hermite_destroy(hermite_ctx* c)
{
    if (!c) return HERMITE_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    drop_graphs(c);
    Buf* bufs[] = {&c->plan, &c->act_start, &c->act_cnt, &c->chunks, &c->item_off,
                   &c->partial, &c->ref_pos, &c->ref_idx, &c->ref_p, &c->ref_tmp,
                   &c->ref_ucnt, &c->ref_ccnt,
                   &c->rplan, &c->ract_start, &c->ract_cnt, &c->rchunks, &c->ritem_off,
                   &c->sel_min, &c->sel_cnt, &c->step_idx, &c->step_na,
                   &c->step_T, &c->step_out, &c->step_acl, &c->phi, &c->counters,
                   &c->ticket, &c->flag, &c->lvl_perm, &c->lvl_tmp, &c->lvl_cnt,
                   &c->lvl_cursor, &c->lvl_misc, &c->lvl_na, &c->lvl_lv, &c->lvl_cst,
                   &c->lvl_ccnt, &c->lvl_ccum, &c->lvl_cna, &c->lvl_bits};
    for (Buf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return HERMITE_OK;
}

int hermite_sync(hermite_ctx* c, void* stream)
{
    CHECK(check_ctx(c));
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    HIP_OK(hipGetLastError());
    return HERMITE_OK;
}

int hermite_select_block(hermite_ctx* c, const hermite_state* s, int32_t* idx_out,
                         int32_t* n_act_dev, int64_t* T_dev, int64_t T_end, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    if (!idx_out || !n_act_dev || !T_dev) return fail(HERMITE_EINVAL, "null output pointer");
    const int nb = select_blocks(s->n);
    CHECK(ensure(c, c->sel_min, sizeof(int64_t) * nb));
    CHECK(ensure(c, c->sel_cnt, sizeof(int32_t) * nb));
    HIP_OK(launch_select(s->n, s->t, s->dt, T_end, idx_out, n_act_dev, T_dev,
                         (int64_t*)c->sel_min.p, (int32_t*)c->sel_cnt.p,
                         (int64_t*)c->counters.p, (hipStream_t)stream));
    return HERMITE_OK;
}

int hermite_predict(hermite_ctx* c, const hermite_state* s, const int64_t* T_dev,
                    int64_t T_host, const int32_t* n_act_dev, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    HIP_OK(launch_predict(s->n, s->tick_bits, s->x, s->v, s->a, s->j, s->t, T_dev, T_host,
                          n_act_dev, s->xp, s->vp, (hipStream_t)stream));
    return HERMITE_OK;
}

int hermite_force_jerk(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                       const int32_t* idx, const int32_t* n_act_dev, int32_t n_act_max,
                       double eps2, int precision, double* acc, double* jerk, double* pot,
                       void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    if (n_act_max < 0 || n_act_max > s->n)
        return fail(HERMITE_EINVAL, "n_act_max = %d out of range [0, n]", n_act_max);
    if (n_act_max == 0) return HERMITE_OK;
    if (!idx && n_act_max != s->n)
        return fail(HERMITE_EINVAL, "identity index list needs n_act_max == n");
    if (!acc || !jerk) return fail(HERMITE_EINVAL, "null output pointer");
    SweepArgs a;
    const hermite_tuning& tu = c->tuning[precision];
    CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, idx, n_act_dev, n_act_max, eps2, precision, tu, acc,
                        jerk, pot, &a));
    return run_force(c, a, precision, tu, false, (hipStream_t)stream);
}

int hermite_force_jerk_timed(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                             const int32_t* idx, int32_t n_act, double eps2, int precision,
                             double* acc, double* jerk, double* pot, int32_t reps,
                             double* ms_out, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    if (n_act < 1 || n_act > s->n) return fail(HERMITE_EINVAL, "n_act = %d out of range [1, n]", n_act);
    if (!idx && n_act != s->n)
        return fail(HERMITE_EINVAL, "identity index list needs n_act == n");
    if (!acc || !jerk || !ms_out) return fail(HERMITE_EINVAL, "null output pointer");
    if (reps < 1) return fail(HERMITE_EINVAL, "reps = %d < 1", reps);
    hipStream_t st = (hipStream_t)stream;
    SweepArgs a;
    const hermite_tuning& tu = c->tuning[precision];
    CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, idx, nullptr, n_act, eps2, precision, tu, acc,
                        jerk, pot, &a));
    SweepArgs ra;
    if (a.refine) CHECK(prepare_refine(c, a, &ra));
    const int grid = std::max(1, c->n_cu * tu.wg_per_cu);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int rc = HERMITE_OK;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 4 && rc == HERMITE_OK; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) rc = fail(HERMITE_EHIP, "hipEventCreate failed");
    for (int r = 0; r < reps && rc == HERMITE_OK; ++r) {
        hipError_t e = hipEventRecord(ev[0], st);
        if (e == hipSuccess)
            e = launch_force(a, a.refine ? &ra : nullptr, precision, tu.variant, grid, false, st,
                             ev + 1);
        if (e == hipSuccess) e = hipEventRecord(ev[3], st);
        if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
        float ms[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]);
        if (e != hipSuccess) {
            rc = fail(HERMITE_EHIP, "timed sweep: %s", hipGetErrorString(e));
            break;
        }
        for (int k = 0; k < 3; ++k) {
            sum[k] += ms[k];
            sum[3] += ms[k];
        }
    }
    for (int k = 0; k < 4; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
    CHECK(rc);
    for (int k = 0; k < 4; ++k) ms_out[k] = sum[k] / reps;
    return HERMITE_OK;
}

int hermite_force_jerk_noalloc(const hermite_state* s, const hermite_clusters* cl,
                               const int32_t* idx, const int32_t* n_act_dev, int32_t n_act_max,
                               double eps2, int precision, double* acc, double* jerk,
                               double* pot, void* stream)
{
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    if (n_act_max < 0 || n_act_max > s->n)
        return fail(HERMITE_EINVAL, "n_act_max = %d out of range [0, n]", n_act_max);
    if (n_act_max > kNoAllocMaxActive)
        return fail(HERMITE_EINVAL,
                    "n_act_max = %d exceeds the allocation-free limit of %lld active particles",
                    n_act_max, (long long)kNoAllocMaxActive);
    if (cl && cl->n_clusters > kNoAllocMaxClusters)
        return fail(HERMITE_EINVAL,
                    "%d clusters exceed the allocation-free limit of %d", cl->n_clusters,
                    kNoAllocMaxClusters);
    if (n_act_max == 0) return HERMITE_OK;
    if (!idx && n_act_max != s->n)
        return fail(HERMITE_EINVAL, "identity index list needs n_act_max == n");
    if (!acc || !jerk) return fail(HERMITE_EINVAL, "null output pointer");
    int device = 0;
    HIP_OK(hipGetDevice(&device));
    NoAllocDevice* nd = nullptr;
    CHECK(noalloc_init(device, &nd));
    const SweepScratch sc = noalloc_carve(nd->base);
    const hermite_tuning tu = default_tuning_for(nd->n_cu);
    SweepArgs a, ra;
    fill_sweep(sc, s, cl, s->xp, s->vp, idx, n_act_dev, n_act_max, eps2, precision, tu,
               default_near_factor(precision), default_fp64_below(precision),
               default_fp64_inter_below(precision), nullptr, acc, jerk, pot, &a);
    if (a.refine) fill_refine(sc, a, &ra);
    const int grid = std::max(1, nd->n_cu * tu.wg_per_cu);
    HIP_OK(launch_force(a, a.refine ? &ra : nullptr, precision, tu.variant, grid, false,
                        (hipStream_t)stream));
    return HERMITE_OK;
}

int hermite_correct(hermite_ctx* c, const hermite_state* s, const int32_t* idx,
                    const int32_t* n_act_dev, int32_t n_act_max, const int64_t* T_dev,
                    int64_t T_host, const double* acc, const double* jerk,
                    const double* pot, const hermite_dt_params* p, double* crit_out,
                    void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_dt(p, s->tick_bits));
    if (n_act_max < 0 || n_act_max > s->n)
        return fail(HERMITE_EINVAL, "n_act_max = %d out of range [0, n]", n_act_max);
    if (n_act_max == 0) return HERMITE_OK;
    if (!idx && n_act_max != s->n)
        return fail(HERMITE_EINVAL, "identity index list needs n_act_max == n");
    if (!acc || !jerk) return fail(HERMITE_EINVAL, "null input pointer");
    CorrectArgs ca;
    std::memset(&ca, 0, sizeof ca);
    ca.n = s->n;
    ca.tick_bits = s->tick_bits;
    ca.idx = idx;
    ca.n_act_dev = n_act_dev;
    ca.n_act_max = n_act_max;
    ca.T_dev = T_dev;
    ca.T_host = T_host;
    ca.xp = s->xp;
    ca.vp = s->vp;
    ca.acc1 = acc;
    ca.jrk1 = jerk;
    ca.pot1 = pot;
    ca.x = s->x;
    ca.v = s->v;
    ca.a = s->a;
    ca.j = s->j;
    ca.pot = s->pot;
    ca.t = s->t;
    ca.dt = s->dt;
    ca.eta = p->eta;
    ca.form = p->form;
    ca.k_min = p->k_min;
    ca.k_max = p->k_max;
    ca.crit_out = crit_out;
    ca.counters = (int64_t*)c->counters.p;
    HIP_OK(launch_correct(ca, (hipStream_t)stream));
    return HERMITE_OK;
}

int hermite_init_dt(hermite_ctx* c, const hermite_state* s, const hermite_dt_params* p,
                    void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_dt(p, s->tick_bits));
    HIP_OK(launch_init_dt(s->n, s->tick_bits, s->a, s->j, s->t, s->dt, p->eta, p->form,
                          p->eta_init, p->k_min, p->k_max, (int64_t*)c->counters.p, (hipStream_t)stream));
    return HERMITE_OK;
}

int hermite_initialize(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                       double eps2, int precision, const hermite_dt_params* p, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    CHECK(check_dt(p, s->tick_bits));
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(launch_copy2(3 * s->n, s->x, s->xp, s->v, s->vp, st));
    SweepArgs a;
    const hermite_tuning& tu = c->tuning[precision];
    CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, nullptr, nullptr, (int32_t)s->n, eps2, precision, tu,
                        s->a, s->j, s->pot, &a));
    CHECK(run_force(c, a, precision, tu, false, st));
    HIP_OK(launch_init_dt(s->n, s->tick_bits, s->a, s->j, s->t, s->dt, p->eta, p->form,
                          p->eta_init, p->k_min, p->k_max, (int64_t*)c->counters.p, st));
    return HERMITE_OK;
}

int hermite_energy(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                   double eps2, double* out_dev, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    if (!out_dev) return fail(HERMITE_EINVAL, "null output pointer");
    hipStream_t st = (hipStream_t)stream;
    CHECK(ensure(c, c->phi, sizeof(double) * s->n));
    double* phi = (double*)c->phi.p;
    SweepArgs a;
    const hermite_tuning& tu = c->tuning[HERMITE_FP64];
    CHECK(prepare_sweep(c, s, cl, s->x, s->v, nullptr, nullptr, (int32_t)s->n, eps2, HERMITE_FP64, tu,
                        phi, nullptr, phi, &a));
    a.counters = nullptr;
    CHECK(run_force(c, a, HERMITE_FP64, tu, true, st));
    HIP_OK(launch_energy_reduce(s->n, cl ? cl->n_clusters : 1, cl ? cl->offsets : nullptr,
                                s->m, s->v, phi, out_dev, st));
    return HERMITE_OK;
}

// Enqueues K consecutive block steps; with use_graph they are captured
// once as one graph (keyed by the step parameters and K) and replayed.
static int launch_steps(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                        double eps2, int precision, const hermite_dt_params* p,
                        int64_t T_end, int use_graph, int K, bool level, void* stream);

int hermite_step(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                 double eps2, int precision, const hermite_dt_params* p, int64_t T_end,
                 int use_graph, void* stream)
{
    return launch_steps(c, s, cl, eps2, precision, p, T_end, use_graph, 1, false, stream);
}

// level: select from the step-size order built by level_init (hermite_run).
static int launch_steps(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                        double eps2, int precision, const hermite_dt_params* p,
                        int64_t T_end, int use_graph, int K, bool level, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    CHECK(check_dt(p, s->tick_bits));
    CHECK(ensure_step_scratch(c, s->n));
    // make sure the sweep scratch exists before any capture
    {
        SweepArgs a;
        double* out = (double*)c->step_out.p;
        CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, (int32_t*)c->step_idx.p,
                            (int32_t*)c->step_na.p, (int32_t)s->n, eps2, precision,
                            c->tuning[precision], out, out + 3 * s->n, out + 6 * s->n, &a));
        SweepArgs ra;
        if (a.refine) CHECK(prepare_refine(c, a, &ra));
    }
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) {
        for (int k = 0; k < K; ++k)
            CHECK(enqueue_step(c, s, cl, eps2, precision, p, T_end, level, st));
        return HERMITE_OK;
    }

    const std::string key = step_key(s, cl, eps2, precision, p, T_end, c->tuning[precision]) +
                            "|K" + std::to_string(K) + (level ? "|L" : "");
    GraphEntry* g = nullptr;
    for (auto& e : c->graphs)
        if (e.key == key) g = &e;
    if (!g) {
        if (c->graphs.size() >= 8) {
            auto& e = c->graphs.front();
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            if (e.graph) (void)hipGraphDestroy(e.graph);
            c->graphs.erase(c->graphs.begin());
        }
        GraphEntry e;
        e.key = key;
        HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = HERMITE_OK;
        for (int k = 0; k < K && rc == HERMITE_OK; ++k)
            rc = enqueue_step(c, s, cl, eps2, precision, p, T_end, level, c->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
        if (rc != HERMITE_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess)
            return fail(HERMITE_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        e.graph = graph;
        hipError_t ei = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(HERMITE_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        c->graphs.push_back(e);
        g = &c->graphs.back();
    }
    HIP_OK(hipGraphLaunch(g->exec, st));
    return HERMITE_OK;
}

// Enqueues the finiteness check of s and reads the flag (synchronises).
static int check_finite(hermite_ctx* c, const hermite_state* s, hipStream_t st, int* bad)
{
    CHECK(ensure(c, c->flag, sizeof(int32_t)));
    HIP_OK(launch_check_finite(s->n, s->x, s->v, s->a, s->j, (int32_t*)c->flag.p, st));
    int32_t h = 0;
    HIP_OK(hipMemcpyAsync(&h, c->flag.p, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *bad = h != 0;
    return HERMITE_OK;
}

int hermite_check_finite(hermite_ctx* c, const hermite_state* s, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    int bad = 0;
    CHECK(check_finite(c, s, (hipStream_t)stream, &bad));
    if (bad) return fail(HERMITE_ENONFINITE, "non-finite position, velocity, acceleration or jerk");
    return HERMITE_OK;
}

int hermite_counters(hermite_ctx* c, int64_t out[6], void* stream)
{
    CHECK(check_ctx(c));
    if (!out) return fail(HERMITE_EINVAL, "null output pointer");
    int64_t h[kCounters];
    HIP_OK(hipMemcpyAsync(h, c->counters.p, sizeof(int64_t) * kCounters,
                          hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    for (int k = 0; k < 6; ++k) out[k] = h[k];
    return HERMITE_OK;
}

int hermite_block_histogram(hermite_ctx* c, int64_t out[33], void* stream)
{
    CHECK(check_ctx(c));
    if (!out) return fail(HERMITE_EINVAL, "null output pointer");
    int64_t h[kCounters];
    HIP_OK(hipMemcpyAsync(h, c->counters.p, sizeof(int64_t) * kCounters,
                          hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    for (int k = 0; k < 33; ++k) out[k] = h[kHistBase + k];
    return HERMITE_OK;
}

int hermite_run(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                double eps2, int precision, const hermite_dt_params* p, int64_t T_end,
                int use_graph, int32_t sync_every, int64_t max_steps, int64_t* steps_out,
                int64_t* interactions_out, int32_t* done_out, void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_dt(p, s->tick_bits));
    if (sync_every < 1) return fail(HERMITE_EINVAL, "sync_every must be >= 1");
    const int64_t dtmax = ((int64_t)1) << (s->tick_bits - p->k_min);
    if (T_end < 0 || T_end % dtmax != 0)
        return fail(HERMITE_EINVAL, "T_end must be a non-negative multiple of 2^(tick_bits-k_min)");
    hipStream_t st = (hipStream_t)stream;
    int64_t c0[5], c1[5];
    CHECK(hermite_counters(c, c0, stream));
    // Select from the step-size order unless the sweep selects itself (one
    // small system) or the clusters do not fit the selection's LDS tables.
    bool level = false;
    if (!(cl == nullptr && s->n <= kFusedSelMax) && (!cl || cl->n_clusters <= kLdsClusters)) {
        CHECK(check_clusters(cl, s->n));
        CHECK(ensure_step_scratch(c, s->n));
        CHECK(level_init(c, s, cl, p, st, &level));
    }
    int64_t launched = 0;
    int32_t done = 0;
    for (;;) {
        int batch = sync_every;
        if (max_steps > 0 && launched + batch > max_steps) batch = (int)(max_steps - launched);
        int k = 0;
        for (; k + kRunGraphSteps <= batch; k += kRunGraphSteps)
            CHECK(launch_steps(c, s, cl, eps2, precision, p, T_end, use_graph, kRunGraphSteps,
                               level, stream));
        for (; k < batch; ++k)
            CHECK(launch_steps(c, s, cl, eps2, precision, p, T_end, use_graph, 1, level,
                               stream));
        launched += batch;
        int64_t T = 0;
        int32_t na = 0;
        HIP_OK(hipMemcpyAsync(&T, c->step_T.p, sizeof T, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(&na, c->step_na.p, sizeof na, hipMemcpyDeviceToHost, st));
        int64_t inconsistent = 0;
        if (level)
            HIP_OK(hipMemcpyAsync(&inconsistent, (int64_t*)c->lvl_misc.p + 4,
                                  sizeof inconsistent, hipMemcpyDeviceToHost, st));
        int bad = 0;
        CHECK(check_finite(c, s, st, &bad));   // synchronises st
        if (inconsistent)
            return fail(HERMITE_EHIP, "block selection: inconsistent step-size order "
                        "(a position out of range was not written)");
        if (bad)
            return fail(HERMITE_ENONFINITE,
                        "non-finite state after block time %lld ticks (e.g. coincident "
                        "particles with zero softening)", (long long)T);
        if (na == 0 || T >= T_end) {
            done = 1;
            break;
        }
        if (max_steps > 0 && launched >= max_steps) break;
    }
    CHECK(hermite_counters(c, c1, stream));
    if (steps_out) *steps_out = c1[0] - c0[0];
    if (interactions_out) *interactions_out = c1[1] - c0[1];
    if (done_out) *done_out = done;
    return HERMITE_OK;
}

int hermite_get_tuning(hermite_ctx* c, int precision, hermite_tuning* out)
{
    if (!c || !out) return fail(HERMITE_EINVAL, "null argument");
    CHECK(check_precision(precision));
    *out = c->tuning[precision];
    return HERMITE_OK;
}

int hermite_set_mixed_policy(hermite_ctx* c, int precision, double near_factor,
                             int64_t fp64_below)
{
    if (!c) return fail(HERMITE_EINVAL, "null context");
    CHECK(check_precision(precision));
    if (precision == HERMITE_FP64)
        return fail(HERMITE_EINVAL, "the FP64 sweep has no mixed-precision policy");
    if (!(near_factor >= 0.0) || std::isinf(near_factor))
        return fail(HERMITE_EINVAL, "near-field radius factor must be finite and >= 0");
    if (fp64_below < 0)
        return fail(HERMITE_EINVAL, "fp64_below must be >= 0");
    if (precision == HERMITE_MIXED_SP && fp64_below != 0)
        return fail(HERMITE_EINVAL, "the paper-faithful mode has no FP64 systems (fp64_below = 0)");
    drop_graphs(c);
    c->near_factor[precision] = near_factor;
    c->fp64_below[precision] = fp64_below;
    return HERMITE_OK;
}

int hermite_set_mixed_small_blocks(hermite_ctx* c, int precision, int64_t fp64_inter_below)
{
    if (!c) return fail(HERMITE_EINVAL, "null context");
    CHECK(check_precision(precision));
    if (precision != HERMITE_MIXED && precision != HERMITE_MIXED_2F)
        return fail(HERMITE_EINVAL, "only MIXED and MIXED_2F sweep small blocks in FP64");
    if (fp64_inter_below < 0) return fail(HERMITE_EINVAL, "fp64_inter_below must be >= 0");
    drop_graphs(c);
    c->fp64_inter_below[precision] = fp64_inter_below;
    return HERMITE_OK;
}

int hermite_get_mixed_small_blocks(hermite_ctx* c, int precision, int64_t* fp64_inter_below)
{
    if (!c || !fp64_inter_below) return fail(HERMITE_EINVAL, "null argument");
    CHECK(check_precision(precision));
    *fp64_inter_below = c->fp64_inter_below[precision];
    return HERMITE_OK;
}

int hermite_get_mixed_policy(hermite_ctx* c, int precision, double* near_factor,
                             int64_t* fp64_below)
{
    if (!c || !near_factor || !fp64_below) return fail(HERMITE_EINVAL, "null argument");
    CHECK(check_precision(precision));
    *near_factor = precision == HERMITE_FP64 ? 0.0 : c->near_factor[precision];
    *fp64_below = precision == HERMITE_FP64 ? 0 : c->fp64_below[precision];
    return HERMITE_OK;
}

int hermite_set_tuning(hermite_ctx* c, int precision, const hermite_tuning* in)
{
    if (!c || !in) return fail(HERMITE_EINVAL, "null argument");
    CHECK(check_precision(precision));
    if (in->wg_per_cu < 1 || in->wg_per_cu > 64 || in->target_lanes < kWG ||
        in->min_j_per_lane < 1 || in->variant < 0 || in->variant > 7)
        return fail(HERMITE_EINVAL, "tuning out of range");
    c->tuning[precision] = *in;
    return HERMITE_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: times candidate launch shapes with HIP events (a screen, then
// interleaved re-timing of the fastest) and keeps the fastest one whose
// output stays within the precision's tolerance of an FP64 sweep.
// ---------------------------------------------------------------------------
namespace {

int64_t pow2_bucket(int64_t v)
{
    int64_t b = 1;
    while (b < v) b <<= 1;
    return b;
}

std::string cache_key(const hermite_ctx* c, int precision, int64_t n, int32_t n_act)
{
    std::ostringstream k;
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    std::string arch = c->arch.substr(0, c->arch.find(':'));
    k << arch << "|hip" << rt << "|p" << precision << "|n" << pow2_bucket(n) << "|a"
      << pow2_bucket(n_act);
    return k.str();
}

// The cache is a JSON object with one entry per line:
//   "key": {"target_lanes": T, "wg_per_cu": W, "min_j_per_lane": M, "variant": V, "us": U,
//           "partial_bytes": B},
// (U: the sweep's median time in microseconds; B: HBM bytes of its j-split
// partial sums, written and read back).
std::map<std::string, std::string> read_cache(const char* path)
{
    std::map<std::string, std::string> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        const size_t b0 = line.find('{', q1 == std::string::npos ? 0 : q1);
        const size_t b1 = line.rfind('}');
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos || b1 < b0)
            continue;
        m[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(b0, b1 - b0 + 1);
    }
    return m;
}

bool field(const std::string& obj, const char* name, double* out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = obj.find(pat);
    if (p == std::string::npos) return false;
    *out = std::strtod(obj.c_str() + p + pat.size(), nullptr);
    return true;
}

int write_cache(const char* path, const std::map<std::string, std::string>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return fail(HERMITE_EINVAL, "cannot write tuning cache %s", path);
        f << "{\n";
        size_t k = 0;
        for (const auto& e : m) {
            f << " \"" << e.first << "\": " << e.second << (++k < m.size() ? ",\n" : "\n");
        }
        f << "}\n";
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return fail(HERMITE_EINVAL, "cannot replace tuning cache %s", path);
    return HERMITE_OK;
}

double max_rel_diff(const std::vector<double>& a, const std::vector<double>& b, int64_t na,
                    int q0, int q1)
{
    // max over particles of |a - b| / |b| for the vector (or scalar) rows
    // q0..q1-1; particles with a zero reference norm compare absolutely.
    double worst = 0.0;
    for (int64_t p = 0; p < na; ++p) {
        double dn = 0.0, rn = 0.0;
        for (int q = q0; q < q1; ++q) {
            const double d = a[q * na + p] - b[q * na + p];
            dn += d * d;
            rn += b[q * na + p] * b[q * na + p];
        }
        const double r = rn > 0.0 ? std::sqrt(dn / rn) : std::sqrt(dn);
        if (!(r <= worst)) worst = r;
    }
    return worst;
}

}  // namespace

extern "C" {

int hermite_autotune(hermite_ctx* c, const hermite_state* s, const hermite_clusters* cl,
                     double eps2, int precision, int32_t n_act, const char* cache_path,
                     void* stream)
{
    CHECK(check_ctx(c));
    CHECK(check_state(s));
    CHECK(check_precision(precision));
    CHECK(check_clusters(cl, s->n));
    if (!cl) CHECK(check_eps2(eps2));
    if (n_act < 1 || n_act > s->n) return fail(HERMITE_EINVAL, "n_act out of range [1, n]");
    hipStream_t st = (hipStream_t)stream;
    CHECK(ensure(c, c->step_idx, sizeof(int32_t) * s->n));
    int32_t* idx = (int32_t*)c->step_idx.p;
    HIP_OK(launch_iota(n_act, idx, st));
    double* out = nullptr;
    HIP_OK(hipMalloc(&out, sizeof(double) * 7 * (size_t)n_act));
    std::vector<double> ref(7 * (size_t)n_act), got(7 * (size_t)n_act);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const hermite_tuning base = default_tuning(c, precision);
    auto run_p = [&](int prec, const hermite_tuning& tu, int reps, double* us,
                     std::vector<double>* res) -> int {
        SweepArgs a;
        CHECK(prepare_sweep(c, s, cl, s->xp, s->vp, idx, nullptr, n_act, eps2, prec, tu, out,
                            out + 3 * (size_t)n_act, out + 6 * (size_t)n_act, &a));
        a.counters = nullptr;
        CHECK(run_force(c, a, prec, tu, false, st));   // warm-up
        HIP_OK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) CHECK(run_force(c, a, prec, tu, false, st));
        HIP_OK(hipEventRecord(e1, st));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        *us = 1000.0 * ms / reps;
        if (res)
            HIP_OK(hipMemcpy(res->data(), out, sizeof(double) * res->size(),
                             hipMemcpyDeviceToHost));
        return HERMITE_OK;
    };
    auto run = [&](const hermite_tuning& tu, int reps, double* us,
                   std::vector<double>* res) -> int {
        return run_p(precision, tu, reps, us, res);
    };
    // Accuracy guard: every candidate is compared with an FP64 sweep of the
    // same particles; it must be as close to it as the tolerance of its
    // precision, or (mixed) as close as the default shape is.
    auto errs = [&](const std::vector<double>& g, const std::vector<double>& r, double e[3]) {
        e[0] = max_rel_diff(g, r, n_act, 0, 3);
        e[1] = max_rel_diff(g, r, n_act, 3, 6);
        e[2] = max_rel_diff(g, r, n_act, 6, 7);
    };
    int rc = HERMITE_OK;
    double best_us = 0.0, partial_bytes = 0.0;
    hermite_tuning best = base;
    std::vector<std::pair<double, hermite_tuning>> passed;   // screened candidates
    const double tol = precision == HERMITE_FP64 ? 1e-13 : 1e-6;
    double limit[3] = {tol, tol, tol};
    std::vector<double> ref64(7 * (size_t)n_act);
    do {
        double us;
        rc = run_p(HERMITE_FP64, default_tuning(c, HERMITE_FP64), 1, &us, &ref64);
        if (rc != HERMITE_OK) break;
        rc = run(base, 3, &us, &ref);
        if (rc != HERMITE_OK) break;
        best_us = us;
        double e[3];
        errs(ref, ref64, e);
        for (int q = 0; q < 3; ++q) limit[q] = std::max(tol, 1.5 * e[q]);
        const std::vector<int> mjs = n_act >= 8192 ? std::vector<int>{4}
                                                   : std::vector<int>{4, 16, 64};
        // variants: particles per lane (bit 0), FP32 difference form (bit 1,
        // MIXED and MIXED_2F), FP32 run length (bit 2, mixed precisions)
        std::vector<int> vars;
        for (int var = 0; var < 8; ++var) {
            if ((var & 2) && precision != HERMITE_MIXED && precision != HERMITE_MIXED_2F)
                continue;
            if ((var & 4) && precision == HERMITE_FP64) continue;
            vars.push_back(var);
        }
        for (int var : vars) {
            if (rc != HERMITE_OK) break;
            for (int w = 2; w <= 8 && rc == HERMITE_OK; ++w) {
                for (int f : {1, 2, 4, 8}) {
                    for (int mj : mjs) {
                        hermite_tuning tu;
                        tu.wg_per_cu = w;
                        tu.target_lanes = c->n_cu * w * kWG * f;
                        tu.min_j_per_lane = mj;
                        tu.variant = var;
                        rc = run(tu, 3, &us, &got);
                        if (rc != HERMITE_OK) break;
                        double ge[3];
                        errs(got, ref64, ge);
                        const bool ok = ge[0] <= limit[0] && ge[1] <= limit[1] &&
                                        ge[2] <= limit[2];
                        if (ok) passed.emplace_back(us, tu);
                    }
                    if (rc != HERMITE_OK) break;
                }
            }
        }
        if (rc != HERMITE_OK) break;
        // A 3-launch screen is noisy, and the minimum over ~100 candidates
        // picks lucky timings: the fastest kFinalists (and the default) are
        // timed again in kRounds interleaved rounds of kFinalReps launches,
        // and the lowest median wins.
        constexpr size_t kFinalists = 6;
        constexpr int kRounds = 3, kFinalReps = 10;
        std::sort(passed.begin(), passed.end(),
                  [](const std::pair<double, hermite_tuning>& x,
                     const std::pair<double, hermite_tuning>& y) { return x.first < y.first; });
        if (passed.size() > kFinalists) passed.resize(kFinalists);
        passed.emplace_back(best_us, base);
        std::vector<std::vector<double>> t(passed.size());
        for (int r = 0; r < kRounds && rc == HERMITE_OK; ++r)
            for (size_t k = 0; k < passed.size() && rc == HERMITE_OK; ++k) {
                rc = run(passed[k].second, kFinalReps, &us, nullptr);
                t[k].push_back(us);
            }
        if (rc != HERMITE_OK) break;
        for (size_t k = 0; k < passed.size(); ++k) {
            std::sort(t[k].begin(), t[k].end());
            const double med = t[k][t[k].size() / 2];
            if (k == 0 || med < best_us) {
                best_us = med;
                best = passed[k].second;
            }
        }
        // the chosen shape's j-split: its partial sums are written to HBM and
        // read back by the reduction (one row set per active particle and
        // j-chunk)
        rc = run(best, 1, &us, nullptr);
        if (rc != HERMITE_OK) break;
        SweepPlan P;
        if (hipMemcpy(&P, c->plan.p, sizeof P, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = fail(HERMITE_EHIP, "reading the sweep plan failed");
            break;
        }
        partial_bytes = 2.0 * (double)P.s_max * kRows * sizeof(double) * (double)P.n_act;
    } while (0);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    CHECK(rc);
    c->tuning[precision] = best;
    if (cache_path) {
        auto m = read_cache(cache_path);
        std::ostringstream o;
        o << "{\"target_lanes\": " << best.target_lanes << ", \"wg_per_cu\": " << best.wg_per_cu
          << ", \"min_j_per_lane\": " << best.min_j_per_lane << ", \"variant\": "
          << best.variant << ", \"us\": " << best_us << ", \"partial_bytes\": "
          << partial_bytes << "}";
        m[cache_key(c, precision, s->n, n_act)] = o.str();
        CHECK(write_cache(cache_path, m));
    }
    return HERMITE_OK;
}

int hermite_load_tuning(hermite_ctx* c, const char* cache_path, int precision, int64_t n,
                        int32_t n_act)
{
    CHECK(check_ctx(c));
    CHECK(check_precision(precision));
    if (!cache_path) return fail(HERMITE_EINVAL, "null cache path");
    const auto m = read_cache(cache_path);
    const auto it = m.find(cache_key(c, precision, n, n_act));
    if (it == m.end()) return fail(HERMITE_EINVAL, "no tuning entry for this device and size");
    double tl, wg, mj, var;
    if (!field(it->second, "target_lanes", &tl) || !field(it->second, "wg_per_cu", &wg) ||
        !field(it->second, "min_j_per_lane", &mj) || !field(it->second, "variant", &var))
        return fail(HERMITE_EINVAL, "malformed tuning entry");
    hermite_tuning t;
    t.target_lanes = (int32_t)tl;
    t.wg_per_cu = (int32_t)wg;
    t.min_j_per_lane = (int32_t)mj;
    t.variant = (int32_t)var;
    return hermite_set_tuning(c, precision, &t);
}

}  // extern "C"
