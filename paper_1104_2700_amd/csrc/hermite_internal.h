// Internal declarations shared by the HIP translation units of libhermite.
// Not part of the public ABI (include/hermite.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

// Workgroup size of the sweep (four wave64s) and the number of j-particles
// staged through LDS per tile (one per thread).
constexpr int kWG = 256;
constexpr int kTJ = 256;

// Device counters: [0] block steps, [1] interactions, [2] clamped steps,
// [3] last block time, [4] last n_act, [5] particles refined in FP64 by a
// mixed sweep, [kHistBase + b] block-size histogram.
constexpr int kHistBase = 8;

// Rows of the sweep's partial sums per (j-chunk, active particle): acc xyz,
// jerk xyz, -pot, and the packed FP32 error estimates of the mixed paths.
constexpr int kRows = 8;
constexpr int kCounters = kHistBase + 33;

// Shape of one force sweep, decided on the device from the active count
// (so that a captured graph adapts to every block size).
struct SweepPlan {
    int32_t n_act;        // active particles this call
    int32_t L;            // lanes cooperating on one active particle
    int32_t ti;           // active particles per work item (kWG / L)
    int32_t s_max;        // largest number of j-chunks of any cluster
    int64_t jc;           // j-chunk length (multiple of kTJ)
    int32_t total_items;  // work items (cluster, i-tile, j-chunk)
    int32_t fp64_all;     // mixed precisions: this block is swept in FP64 (its
                          // interactions are below SweepArgs::fp64_inter_below)
};

// Everything the plan, sweep and reduce kernels read.  Passed by value.
struct SweepArgs {
    const double* xp;          // [3][n] positions of i and j
    const double* vp;          // [3][n] velocities of i and j
    const double* m;           // [n]
    int64_t n;
    const int32_t* idx;        // [n_act_max] or null (identity)
    const int32_t* n_act_dev;  // or null (n_act_max)
    int32_t n_act_max;
    int32_t n_clusters;        // >= 1
    const int64_t* offsets;    // [C+1] or null when C == 1
    const double* eps2_c;      // [C] or null when C == 1
    double eps2;               // used when eps2_c is null
    int64_t n_cmax;            // largest cluster size
    // plan and per-cluster scratch (device)
    SweepPlan* plan;
    int32_t* act_start;        // [C]
    int32_t* act_cnt;          // [C]
    // Block-step path with clusters: the selection writes act_start (for
    // every cluster that starts below n) and the cluster of every active
    // position, so neither the plan nor the reduction searches.
    int32_t* act_cluster;      // [n_act_max] or null
    int32_t sel_clusters;      // nonzero: act_start / act_cluster come from the selection
    int32_t* chunks;           // [C]
    int32_t* item_off;         // [C+1]
    double* partial;           // [s_max][7][n_act]
    int64_t partial_cap;       // doubles available in partial
    // tuning
    int32_t target_lanes;
    int32_t min_j_per_lane;
    int32_t ipl;               // active particles per lane (set by launch_force)
    int32_t one_chunk;         // nonzero: no j-split across work items (the
                               // paper-faithful mode's FP32 jerk sums span all j)
    // mixed precisions: pairs closer than near_factor * N_c^(-1/3) (N_c the
    // size of the particle's system) are summed in FP64, and systems with
    // N_c < fp64_below are swept in FP64 altogether
    double near_factor;
    int64_t fp64_below;
    // mixed precisions: blocks of fewer interactions than this are swept in
    // FP64 (latency-bound there, where the refinement's launches would cost
    // more than FP32 arithmetic saves); 0: never
    int64_t fp64_inter_below;
    // nonzero: the reduce stage flags particles whose estimated mixed
    // error is too large (ref_pos[p] = 1) and plans their FP64 refinement
    int32_t refine;
    // with refinement: a block the plan puts in FP64 (fp64_all) is swept by
    // the refine sweep's launch, with the whole block as its list, and its
    // sums taken from there by the corrector (block steps) or the scatter
    // (force calls); no other sweep launch and not the flagging reduce touch it
    int32_t defer_fp64;
    int32_t* ref_pos;          // [n_act_max] a flagged position's slot in the list, or -1
    int32_t* ref_idx;          // [n_act_max] flagged particles (the refine sweep's idx)
    int32_t* ref_p;            // [n_act_max] their active positions
    int32_t* ref_tmp;          // [n_act_max] flagged positions, compacted per reduce unit
    int32_t* ref_ucnt;         // [n_act_max / 4 + 1] flagged per reduce unit, then its first slot
    int32_t* ref_ccnt;         // [C] flagged per cluster, then placement cursors
    // items a sweep launch takes: 0 all; 1 the mixed kernel's: systems with
    // N_c >= fp64_below in a block the plan has not put in FP64 (fp64_all);
    // 2 the FP64 kernel's: the others
    int32_t kind;
    // counters (may be null): [0] steps, [1] interactions, [4] last n_act
    int64_t* counters;
    // On-the-fly prediction (block-step path): when pred_x is non-null the
    // i and j particles are predicted from pred_x/v/a/j at block time
    // *pred_T from their times pred_t (equations (xpred), (vpred)) instead
    // of being read from xp, vp.
    const double* pred_x;
    const double* pred_v;
    const double* pred_a;
    const double* pred_j;
    const int64_t* pred_t;
    const int64_t* pred_T;
    double tick;               // 2^-tick_bits
    // Selection fused into the sweep (one system of n <= kSelBlock, block
    // step path): every workgroup takes the block time and the active list
    // from t (pred_t) and sel_dt itself; workgroup 0 publishes the list,
    // n_act, T, the plan and the counters for the corrector.
    const int64_t* sel_dt;
    int64_t sel_T_end;
    int32_t* sel_idx_out;      // [n]
    int32_t* sel_na_out;
    int64_t* sel_T_out;
    // outputs of the reduce stage
    double* acc;               // [3][n_act_max]
    double* jerk;              // [3][n_act_max] or null
    double* pot;               // [n_act_max] or null
};

// Cluster tables up to this many entries are staged in LDS by the kernels
// that search them (offsets in the selection, item offsets in the sweep).
constexpr int kLdsClusters = 2048;

// Grid of the grid-stride reduce/correct kernels: enough blocks for one
// wave per particle (the many-chunk mode), capped at 4096 blocks; the
// kernels loop over the rest, and the one-thread-per-particle mode uses
// the same grid.
inline int reduce_grid(int64_t n_act_max)
{
    const int64_t g = (n_act_max + (kWG / 64) - 1) / (kWG / 64);
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// Sweep launchers (sweep.hip).  precision: 0 fp64, 1 mixed, 2 mixed-2f,
// 3 mixed with FP32 velocities and jerk sums.
// variant bit 0: two active particles per lane (else one); bit 1: split
// FP32 hi/lo differences in the mixed precisions.
// pot_only: the energy sweep (FP64, potential only).
// ra (or null): the refine sweep of a mixed sweep with refinement (a.refine):
// the reduce flags and plans, the FP64 refine sweep runs, and the refined
// sums are scattered into the outputs.
// marks (or null): two events recorded on st after the plan kernel and after
// the sweep kernel(s), so that each phase can be timed on its own stream.
hipError_t launch_force(const SweepArgs& a, const SweepArgs* ra, int precision, int variant,
                        int grid, bool pot_only, hipStream_t st,
                        const hipEvent_t* marks = nullptr);

// Block-step form of the refinement: the flagging reduce into the compact
// outputs a.acc / a.jerk / a.pot, then the FP64 refine sweep (the corrector,
// launch_correct_refine, takes the refined sums of flagged positions).
hipError_t launch_reduce_refine(const SweepArgs& a, const SweepArgs& ra, int variant, int grid,
                                hipStream_t st);

// Block selection (integrate.hip).
// Number of select blocks (size of block_min / block_cnt) for n particles.
int select_blocks(int64_t n);

hipError_t launch_select(int64_t n, const int64_t* t, const int64_t* dt,
                         int64_t T_end, int32_t* idx, int32_t* n_act,
                         int64_t* T, int64_t* block_min, int32_t* block_cnt,
                         int64_t* counters, hipStream_t st);

hipError_t launch_predict(int64_t n, int tick_bits, const double* x,
                          const double* v, const double* a, const double* j,
                          const int64_t* t, const int64_t* T_dev,
                          int64_t T_host, const int32_t* n_act_dev,
                          double* xp, double* vp, hipStream_t st);

struct CorrectArgs {
    int64_t n;
    int tick_bits;
    const int32_t* idx;
    const int32_t* n_act_dev;
    int32_t n_act_max;
    const int64_t* T_dev;
    int64_t T_host;
    const double* xp;
    const double* vp;
    const double* acc1;        // [3][n_act_max]
    const double* jrk1;        // [3][n_act_max]
    const double* pot1;        // [n_act_max] or null
    double* x;
    double* v;
    double* a;
    double* j;
    double* pot;
    int64_t* t;
    int64_t* dt;
    double eta;
    int form;
    int k_min;
    int k_max;
    double* crit_out;          // or null
    int64_t* counters;         // [2] += clamped, or null
    int predict_i;             // 1: predict the active particle from x, v, a, j, t
                               //    at T instead of reading xp, vp
    int32_t* na_seen;          // or null: receives n_act (a run's selection reads the
                               // previous block's size from here, never from a word it
                               // rewrites itself)
    uint8_t* lv_out;           // [n_act_max] or null: log2 of each position's new step
};

hipError_t launch_correct(const CorrectArgs& c, hipStream_t st);
hipError_t launch_correct_refine(const CorrectArgs& c, const SweepArgs& a, const SweepArgs& ra,
                                 hipStream_t st);

// Fused block-step stages: selection and the sweep plan in two launches
// (prediction is folded into the sweep and the corrector), and the
// corrector with the fixed-order reduction of the sweep's partial sums.
hipError_t launch_step_select(int64_t n, const int64_t* t, const int64_t* dt, int64_t T_end,
                              int32_t* idx, int32_t* n_act, int64_t* T, int64_t* block_min,
                              int32_t* block_cnt, int64_t* counters, uint32_t* ticket,
                              const SweepArgs& sa, hipStream_t st);
// Largest system whose sweep workgroups select the block themselves: every
// workgroup reads all t, dt, so the fusion pays only while that read is
// small (measured: faster at 1024 and 2048, slower at 4096).
constexpr int kFusedSelMax = 2048;

// Largest number of work items the plan gives for any active count of a
// single system (host; sizes the grid of the fused select + sweep launch).
int max_plan_items(const SweepArgs& a);

// Selection fused into the sweep (sel_* fields of a set, n <= kFusedSelMax,
// one system).
hipError_t launch_select_sweep(const SweepArgs& a, int precision, int variant, int grid,
                               hipStream_t st);

hipError_t launch_sweep_only(const SweepArgs& a, int precision, int variant, int grid,
                             hipStream_t st);

// Step-size structure of a block-step run.  Every t_i is a multiple of its
// power-of-two step dt_i and t_i <= T_last < t_i + dt_i (T_last: the last
// block time), so particle i's next time is the first multiple of dt_i
// after T_last.  The next block time is then the first multiple of the
// smallest occupied step after T_last, and the active block is every
// particle whose step divides it: with the particles ordered by step size
// (perm), a prefix of perm.  The corrector gives every active particle a
// step that divides the block time, so re-sorting that prefix by the new
// steps keeps the whole order; selection costs O(n_act) instead of O(n).
struct LevelArgs {
    int64_t n;
    const int64_t* t;
    const int64_t* dt;
    int64_t dt_floor;    // smallest step the corrector can give, 2^(tick_bits - k_max)
    int32_t* perm;       // [n] particle ids by step size, smallest first (ensembles:
                         // within each cluster's range)
    int32_t* cnt;        // [64] particles with dt = 2^b ticks (of the whole ensemble)
    int32_t* cursor;     // [64] (building the order)
    int64_t* misc;       // [0] T_last; [1] max t, [2] min t + dt, [3] inconsistent (checks);
                         // [4] a position out of range was not written
    int32_t* tmp;        // [n] re-sort scratch for blocks beyond the LDS staging
    int32_t* na_prev;    // the previous block's n_act, written by the corrector
    uint32_t* bits;      // [(n + 31) / 32] active-particle bitmap (zeroed once, left zero)
    int64_t T_end;
    int32_t* na;         // n_act: the previous step's in, this step's out
    int64_t* T;          // block time: the previous step's in, this step's out
    int32_t* idx;        // [n] active list grouped by cluster (C > 1)
    const uint8_t* lv;   // [n] log2 of the new step of every position of the last block
                         // (written by the corrector): the re-sort reads these in
                         // position order instead of gathering dt through perm
    int64_t* counters;
    // ensembles (C > 1): per-cluster step-size orders
    int32_t n_clusters;
    const int64_t* offsets;  // [C + 1]
    int32_t* ccnt;       // [C][64] particles of cluster c with dt = 2^b ticks
    int32_t* ccum;       // [C][64] their running sums over b (steps <= 2^b)
    int32_t* cna;        // [C] size of cluster c's last block
    int32_t* cst;        // [C] its first position in the last block's list
};

// Counts the steps of a state and checks that it is one the block scheme
// can have produced (misc[1..3]); misc and cnt must hold {0, INT64_MIN,
// INT64_MAX, 0} and zeros.  launch_level_build then orders the particles
// (cursor zeroed; ensembles: per cluster) and sets T_last = max t and
// *na = *na_prev = 0.
hipError_t launch_level_count(const LevelArgs& L, hipStream_t st);
hipError_t launch_level_build(const LevelArgs& L, hipStream_t st);
// Re-sorts the previous block by its new steps, selects the next block,
// lists it (ensembles: grouped by cluster, C <= kLdsClusters) and plans the
// sweep.  One system: one workgroup.  Ensembles: two kernels, a re-sort
// with one workgroup per cluster, then the selection, in which every
// workgroup derives the block from the same tables and lists the blocks of
// its clusters; no workgroup waits on another.
hipError_t launch_level_select(const LevelArgs& L, const SweepArgs& sa, hipStream_t st);
hipError_t launch_correct_reduce(const CorrectArgs& c, const SweepArgs& sa, hipStream_t st);

hipError_t launch_init_dt(int64_t n, int tick_bits, const double* a,
                          const double* j, int64_t* t, int64_t* dt,
                          double eta, int form, double eta_init, int k_min, int k_max,
                          int64_t* counters, hipStream_t st);

hipError_t launch_copy2(int64_t count, const double* src0, double* dst0,
                        const double* src1, double* dst1, hipStream_t st);

hipError_t launch_iota(int32_t count, int32_t* out, hipStream_t st);

// Clears *flag, then sets it when any x, v, a, j value of the state is not
// finite (not graph-safe: clears with hipMemsetAsync).
hipError_t launch_check_finite(int64_t n, const double* x, const double* v, const double* a,
                               const double* j, int32_t* flag, hipStream_t st);

int sweep_occupancy(int precision, int variant, bool pot_only);

hipError_t launch_energy_reduce(int64_t n, int n_clusters,
                                const int64_t* offsets, const double* m,
                                const double* v, const double* phi,
                                double* out, hipStream_t st);

}  // namespace hm
