"""Whole-run workloads on one GPU (block-timestep integrations).

    python -m paper_1104_2700_amd.workloads <name> [--t-end T] [--start-div D] [--out file.json]

(--start-div D: first steps eta_f/D |a|/|j| instead of eta_f |a|/|j|; the
start-up rule is a reading, and the default factor lets the first step
dominate a short run's energy error.)

Names:
  c1  Plummer N = 1024, eps = 1/64, eta = 0.02, FP64, t = 0 -> 0.125
  c2  Plummer N = 16384, eps = 4/N, FP64: full sweep, and a block run to t = 1
      with the histogram of active-block sizes
  c3  Plummer N = 65536, eps = 4/N: sweep time vs active count (both
      precisions) and a mixed-precision block run with its energy drift
  c4  256 independent Plummer clusters (N_c log-uniform in [256, 8192],
      eps_c = 4/N_c), mixed precision: the batched ensemble (one persistent
      sweep launch per block step, graph-replayed steps, autotuned shape)
      against a serial loop over the clusters
  c5  Plummer N = 131072 with a Salpeter mass spectrum and 10 % binaries,
      eps = 1e-5, two-float accumulation, t = 0 -> 0.25
  e1  force and jerk error of the reduced-precision sweeps against the FP64
      sweep as N grows (Plummer, eps = 4/N, 1K .. 256K), and the full-sweep
      time of each precision: the cost of summing the jerk in FP64 instead
      of FP32 (Section 3.2)
  e2  energy conservation of block runs with the jerk summed in FP64
      (mixed) and in FP32 (mixed_sp), Plummer N = 256K, t = 0 -> 0.125
  e3  energy error against the number of steps per crossing time, N = 1K,
      FP64, mixed and FP32-jerk forces (the paper's Section 4 energy study)
  e4  whole-run speed against N (Plummer N = 1K .. 16K, eps = 4/N, t = 0 -> 1,
      FP64 and mixed): the paper's Section 5 performance sweep
  o1  HBM bandwidth of the O(N) stages at large N (2^20 .. 2^24 particles):
      standalone select, predict and correct (all particles active)

Every run reports wall time, block steps, interactions, interactions/s,
GFLOPS at the paper's 60 flops per interaction (Section 5), clamped steps
and the relative energy change (energies from FP64 potential sweeps at the
synchronised start and end, Section 4).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import hermite as H
from . import inputs

TB = 20          # time tick 2^-20
START_DIV = 0    # start-up factor = steady factor / START_DIV (0: the steady factor)
FORMS = {"paper": H.DT_PAPER, "aarseth": H.DT_AARSETH}
K_MIN, K_MAX = 3, 20
RUN_FORM = H.DT_PAPER   # criterion form of the c1-c5 and e2 runs (the --form option)
RUN_PREC = {}           # precision override of the c1-c5 runs (the --precision option)


def _prec(default):
    return RUN_PREC.get("p", default)


def _params(eta, form=None):
    """Timestep parameters of the whole-run workloads (k in [K_MIN, K_MAX]);
    the criterion form follows RUN_FORM and the start-up factor START_DIV
    (the --form and --start-div options)."""
    form = RUN_FORM if form is None else form
    eta_f = eta if form == H.DT_PAPER else math.sqrt(eta)
    return H.dt_params(eta, form, K_MIN, K_MAX,
                       eta_init=(eta_f / START_DIV) if START_DIV else 0.0)


def _log(msg):
    print(msg, flush=True)


def _energy(ctx, s, eps2, clusters=None):
    e = ctx.energy(s, eps2, clusters=clusters).cpu().numpy()
    return e[:, 0] + e[:, 1]


MAX_WALL = 0.0   # seconds; 0: no limit (the --max-wall option)


def block_run(ctx, s, eps2, params, t_end, precision, clusters=None,
              chunk=20000, label=""):
    """Integrates an initialised state to t_end (time units), printing a
    progress line every `chunk` launched steps; with MAX_WALL set, stops
    after the first chunk that ends past it (the stats then cover the time
    reached, t_reached).  Returns a dict of stats."""
    T_end = int(round(t_end * (1 << TB)))
    e0 = _energy(ctx, s, eps2, clusters)
    c0 = ctx.counters()
    h0 = np.array(ctx.block_histogram())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = inter = 0
    t_reached = t_end
    while True:
        st, it, done = ctx.run(s, eps2, params, T_end, precision, use_graph=True,
                               sync_every=256, clusters=clusters, max_steps=chunk,
                               with_done=True)
        steps += st
        inter += it
        cnt = ctx.counters()
        _log("  %s t = %.9f  block steps %d  interactions %.3e  %.1f s"
             % (label, cnt["T"] / (1 << TB), steps, inter, time.perf_counter() - t0))
        if done:
            break
        if MAX_WALL and time.perf_counter() - t0 > MAX_WALL:
            t_reached = cnt["T"] / (1 << TB)
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = ctx.counters()
    hist = (np.array(ctx.block_histogram()) - h0).tolist()
    # a run stopped early has no synchronised state to take the energy of
    rel = np.abs((_energy(ctx, s, eps2, clusters) - e0) / e0) if t_reached == t_end else None
    lv = TB - np.log2(s.dt.cpu().numpy()).astype(np.int64)
    return {
        "dt_levels_final": {int(k): int(c) for k, c in enumerate(np.bincount(lv)) if c},
        "t_end": t_end, "t_reached": t_reached, "wall_s": wall, "block_steps": steps,
        "interactions": inter,
        "interactions_per_s": inter / wall, "gflops_60": 60.0 * inter / wall / 1e9,
        "clamped_steps": c1["clamped"] - c0["clamped"],
        "energy_rel_change_max": float(rel.max()) if rel is not None else None,
        "energy_rel_change_median": float(np.median(rel)) if rel is not None else None,
        "E0": float(e0.sum()) if e0.size == 1 else None,
        "active_size_histogram_log2": {("0" if b == 0 else "[2^%d,2^%d)" % (b - 1, b)): v
                                       for b, v in enumerate(hist) if v},
        # one system: interactions / (steps * n) is the mean block size; an
        # ensemble's interactions weight each cluster's block by its size
        "mean_active": inter / max(steps, 1) / s.n if clusters is None else None,
        "mean_interactions_per_step": inter / max(steps, 1),
    }


class _fp32_mixed:
    """Within the block, MIXED and MIXED_2F sweep every system and every
    block with FP32 pair arithmetic (near field and refinement kept), as
    the accuracy studies need; the policies are restored afterwards."""

    def __init__(self, ctx):
        self.ctx = ctx

    def __enter__(self):
        self.saved = {p: (self.ctx.get_mixed_policy(p), self.ctx.get_mixed_small_blocks(p))
                      for p in (H.MIXED, H.MIXED_2F)}
        for p, ((near, _), _) in self.saved.items():
            self.ctx.set_mixed_policy(p, near, 0)
            self.ctx.set_mixed_small_blocks(p, 0)
        return self

    def __exit__(self, *exc):
        for p, ((near, below), small) in self.saved.items():
            self.ctx.set_mixed_policy(p, near, below)
            self.ctx.set_mixed_small_blocks(p, small)
        return False


def sweep_time(ctx, s, eps2, precision, idx=None, reps=10):
    acc, jrk, pot = ctx.force_jerk(s, idx, eps2, precision)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.force_jerk(s, idx, eps2, precision, acc=acc, jerk=jrk, pot=pot)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _plummer_state(n, seed):
    x, v, m = inputs.plummer(n, seed)
    return H.State(x, v, m, TB)


def c1(ctx, t_end=0.125):
    s = _plummer_state(1024, 1)
    eps2 = (1.0 / 64) ** 2
    p = _params(0.02)
    ctx.initialize(s, eps2, p, H.FP64)
    return {"config": "plummer_n1024_fp64", "run": block_run(ctx, s, eps2, p, t_end, H.FP64,
                                                             label="c1")}


def c2(ctx, t_end=1.0):
    n = 16384
    s = _plummer_state(n, 2)
    eps2 = (4.0 / n) ** 2
    p = _params(0.02)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    ms = sweep_time(ctx, s, eps2, H.FP64)
    ctx.initialize(s, eps2, p, H.FP64)
    run = block_run(ctx, s, eps2, p, t_end, H.FP64, label="c2")
    return {"config": "plummer_n16384_fp64",
            "full_sweep": {"ms": ms, "interactions_per_s": n * n / (ms * 1e-3),
                           "gflops_60": 60 * n * n / (ms * 1e-3) / 1e9},
            "run": run}


def c3(ctx, t_end=1.0, tune_cache=None, run=True):
    """Sweep time against the active count (both precisions; with
    tune_cache, each point at the launch shape the autotuner picks for that
    count, kept in that cache), then a mixed-precision block run."""
    n = 65536
    s = _plummer_state(n, 3)
    eps2 = (4.0 / n) ** 2
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    curve = []
    na = 1
    saved = {p: ctx.get_tuning(H.PRECISIONS[p]) for p in ("fp64", "mixed")}
    while na <= n:
        idx = torch.arange(0, n, n // na, dtype=torch.int32, device="cuda")[:na].contiguous()
        row = {"n_act": na}
        for pname in ("fp64", "mixed"):
            prec = H.PRECISIONS[pname]
            if tune_cache:
                ctx.autotune(s, eps2, prec, na, cache_path=tune_cache)
                row[pname + "_tuning"] = ctx.get_tuning(prec).as_dict()
            ms = sweep_time(ctx, s, eps2, prec, idx, reps=20)
            row[pname + "_us"] = 1e3 * ms
            row[pname + "_interactions_per_s"] = na * n / (ms * 1e-3)
        curve.append(row)
        _log("  c3 n_act %6d  fp64 %.1f us  mixed %.1f us" % (na, row["fp64_us"], row["mixed_us"]))
        na *= 2
    for pname, t in saved.items():
        ctx.set_tuning(H.PRECISIONS[pname], t)
    out = {"config": "plummer_n65536_mixed", "latency_curve": curve, "tuned": bool(tune_cache)}
    if tune_cache:
        with open(tune_cache) as f:
            out["tuning_cache"] = json.load(f)
    if not run:
        return out
    p = _params(0.02)
    prec = _prec(H.MIXED)
    ctx.initialize(s, eps2, p, prec)
    out["run"] = block_run(ctx, s, eps2, p, t_end, prec, label="c3")
    return out


def c4(ctx, t_end=0.5, serial_t_end=0.125, n_clusters=256, serial_clusters=16):
    """Batched ensemble run, then batched vs serial on a subset of clusters."""
    x, v, m, off, eps = inputs.ensemble(n_clusters, 4)
    eps2 = eps ** 2
    sizes = np.diff(off)
    p = _params(0.02)
    out = {"config": "ensemble_%d_clusters_mixed" % n_clusters,
           "n_total": int(off[-1]), "sum_Nc2": float(np.sum(sizes.astype(float) ** 2)),
           "sizes_min_max": [int(sizes.min()), int(sizes.max())]}
    cl = H.Clusters(off, eps2)
    s = H.State(x, v, m, TB)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    prec = _prec(H.MIXED)
    out["tuning"] = ctx.autotune(s, 0.0, prec, int(off[-1]), clusters=cl).as_dict()
    ctx.initialize(s, 0.0, p, prec, clusters=cl)
    out["batched"] = block_run(ctx, s, 0.0, p, t_end, prec, clusters=cl, label="c4 batched")
    # the same clusters, one system at a time, against the batched ensemble
    # of those clusters (a subset keeps the serial loop short)
    if serial_t_end and serial_clusters > 0:
        k = min(serial_clusters, n_clusters)
        hi_all = int(off[k])
        sub_off = off[:k + 1]
        cls = H.Clusters(sub_off, eps2[:k])
        sb = H.State(x[:, :hi_all], v[:, :hi_all], m[:hi_all], TB)
        ctx.initialize(sb, 0.0, p, H.MIXED, clusters=cls)
        bs = block_run(ctx, sb, 0.0, p, serial_t_end, H.MIXED, clusters=cls,
                       label="c4 batched(subset)")
        torch.cuda.synchronize()
        T_end = int(round(serial_t_end * (1 << TB)))
        t0 = time.perf_counter()
        steps = inter = 0
        for c in range(k):
            lo, hi = int(off[c]), int(off[c + 1])
            sc = H.State(x[:, lo:hi], v[:, lo:hi], m[lo:hi], TB)
            ctx.initialize(sc, float(eps2[c]), p, H.MIXED)
            st, it = ctx.run(sc, float(eps2[c]), p, T_end, H.MIXED, use_graph=True,
                             sync_every=256)
            steps += st
            inter += it
            _log("  c4 serial: cluster %d/%d done, %.1f s" % (c + 1, k, time.perf_counter() - t0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out["subset"] = {"clusters": k, "t_end": serial_t_end, "batched": bs,
                         "serial": {"wall_s": wall, "block_steps": steps, "interactions": inter,
                                    "interactions_per_s": inter / wall,
                                    "gflops_60": 60 * inter / wall / 1e9},
                         "batched_vs_serial_speedup": wall / bs["wall_s"]}
    return out


def c5(ctx, t_end=0.25):
    n = 131072
    x, v, m = inputs.plummer_imf_binaries(n, 5)
    s = H.State(x, v, m, TB)
    eps2 = 1e-5 ** 2
    p = _params(0.02)
    prec = _prec(H.MIXED_2F)
    ctx.initialize(s, eps2, p, prec)
    return {"config": "plummer_imf_binaries_n131072_mixed2f",
            "run": block_run(ctx, s, eps2, p, t_end, prec, label="c5")}


def e3(ctx, t_end=0.375, etas=(0.0025, 0.005, 0.01, 0.02, 0.04, 0.08), n=1024, seed=1,
       form="paper"):
    """Energy error against steps per crossing time (Section 4 energy study):
    Plummer N = 1K, eps = 4/N, FP64, mixed and FP32-jerk forces, several
    eta, with the criterion as printed (form "paper": eta sqrt(R)) or in
    its classic form ("aarseth": sqrt(eta R)); the error is averaged over
    the sync times 1/8, 2/8, 3/8 (potential energy from FP64 sweeps);
    start-up factor eta_f/16.  The mixed modes sweep this small system in
    FP32 (the default policy would take FP64 below 8192 particles and for
    blocks below 5e7 interactions): mixed with its FP64 near field and
    refinement, mixed_sp as printed.  n_step =
    particle steps per particle per crossing time (2 sqrt 2 in N-body
    units)."""
    x, v, m = inputs.plummer(n, seed)
    eps2 = (4.0 / n) ** 2
    rows = []
    dform = FORMS[form]
    fp32 = _fp32_mixed(ctx).__enter__()
    for prec_name in ("fp64", "mixed", "mixed_sp"):
        prec = H.PRECISIONS[prec_name]
        for eta in etas:
            s = H.State(x, v, m, TB)
            # start-up factor eta_f/16: with the steady factor the first step
            # dominates the error over 3/8 time units (the scheme's error,
            # not the start-up, is what the study measures)
            eta_f = eta if dform == H.DT_PAPER else math.sqrt(eta)
            p = H.dt_params(eta, dform, K_MIN, K_MAX, eta_init=eta_f / 16)
            ctx.initialize(s, eps2, p, prec)
            e0 = _energy(ctx, s, eps2)[0]
            errs, inter, steps = [], 0, 0
            t0 = time.perf_counter()
            nsync = int(round(t_end * 8))
            for k in range(1, nsync + 1):
                st, it = ctx.run(s, eps2, p, k << (TB - 3), prec, use_graph=True,
                                 sync_every=256)
                steps += st
                inter += it
                errs.append(abs((_energy(ctx, s, eps2)[0] - e0) / e0))
            wall = time.perf_counter() - t0
            n_step = inter / n / n * (2.0 * math.sqrt(2.0) / t_end)
            # final step levels: count of particles with dt = 2^-k, k = 0..TB
            lv = TB - np.log2(s.dt.cpu().numpy()).astype(np.int64)
            levels = np.bincount(lv, minlength=TB + 1).tolist()
            rows.append({"precision": prec_name, "eta": eta, "n_step": n_step,
                         "mean_rel_energy_error": float(np.mean(errs)),
                         "rel_energy_error_at_sync": [float(e) for e in errs],
                         "block_steps": steps, "wall_s": wall, "dt_levels_final": levels})
            _log("  e3 %-8s eta %.4f  n_step %9.1f  <|dE/E|> %.3e  %.1f s" %
                 (prec_name, eta, n_step, np.mean(errs), wall))
    # slope of log error vs log n_step for FP64 over the converging part
    # (errors in [1e-13, 1e-6): larger ones leave the asymptotic regime,
    # smaller ones reach the FP64 rounding floor)
    # (and per precision: the slope over its rows above 1e-9 and 4x its
    # smallest error, i.e. before its floor, and that floor)
    f = [r for r in rows if r["precision"] == "fp64"
         and 1e-13 <= r["mean_rel_energy_error"] < 1e-6]
    ln = np.log([r["n_step"] for r in f])
    le = np.log([r["mean_rel_energy_error"] for r in f])
    slope = float(np.polyfit(ln, le, 1)[0]) if len(f) > 1 else None
    per = {}
    for prec_name in ("fp64", "mixed", "mixed_sp"):
        rs = [r for r in rows if r["precision"] == prec_name]
        floor = min(r["mean_rel_energy_error"] for r in rs)
        fit = [r for r in rs if r["mean_rel_energy_error"] > max(1e-9, 4 * floor)]
        sl = (float(np.polyfit(np.log([r["n_step"] for r in fit]),
                               np.log([r["mean_rel_energy_error"] for r in fit]), 1)[0])
              if len(fit) > 1 else None)
        per[prec_name] = {"floor": floor, "slope_above_floor": sl, "rows_in_fit": len(fit)}
    fp32.__exit__(None, None, None)
    return {"config": "energy_vs_nstep_plummer_n%d" % n, "t_end": t_end, "form": form,
            "rows": rows, "fp64_loglog_slope": slope, "per_precision": per}


def e1(ctx, ns=(1024, 4096, 16384, 65536, 262144), sample=4096, seed=5):
    """Accuracy and cost of the precision modes against N (Section 3.2).

    For each N: a sample of up to `sample` particles evenly spread over the
    index range; per-particle relative errors |f - f64| / |f64| of the
    acceleration and the jerk of each reduced-precision sweep against the
    FP64 sweep (median, 99th percentile, max), and the full-sweep time
    (n_act = N) of every precision; the mixed precisions sweep every N
    with FP32 pair arithmetic here."""
    with _fp32_mixed(ctx):
        return _e1(ctx, ns, sample, seed)


def _e1(ctx, ns, sample, seed):
    rows = []
    for n in ns:
        x, v, m = inputs.plummer(n, seed)
        s = H.State(x, v, m, TB)
        s.xp.copy_(s.x)     # the sweep reads the predicted arrays
        s.vp.copy_(s.v)
        eps2 = (4.0 / n) ** 2
        k = min(sample, n)
        idx = torch.from_numpy((np.arange(k, dtype=np.int64) * n // k).astype(np.int32)).cuda()
        ref_a, ref_j, _ = ctx.force_jerk(s, idx, eps2, H.FP64)
        ref_a, ref_j = ref_a.cpu().numpy(), ref_j.cpu().numpy()
        row = {"n": n, "sample": k, "errors": {}, "sweep_ms": {}}
        for pname in ("mixed", "mixed2f", "mixed_sp"):
            a, j, _ = ctx.force_jerk(s, idx, eps2, H.PRECISIONS[pname])
            a, j = a.cpu().numpy(), j.cpu().numpy()
            ea = np.linalg.norm(a - ref_a, axis=0) / np.linalg.norm(ref_a, axis=0)
            ej = np.linalg.norm(j - ref_j, axis=0) / np.linalg.norm(ref_j, axis=0)
            row["errors"][pname] = {
                "acc": [float(np.median(ea)), float(np.percentile(ea, 99)), float(ea.max())],
                "jerk": [float(np.median(ej)), float(np.percentile(ej, 99)), float(ej.max())]}
        reps = max(2, min(50, int(4e10 / (n * n))))
        for pname in ("fp64", "mixed", "mixed2f", "mixed_sp"):
            ms = sweep_time(ctx, s, eps2, H.PRECISIONS[pname], reps=reps)
            row["sweep_ms"][pname] = ms
        rows.append(row)
        _log("  e1 N %7d  jerk rel err median mixed %.2e  mixed_sp %.2e  "
             "sweep ms fp64 %.3f mixed %.3f mixed_sp %.3f"
             % (n, row["errors"]["mixed"]["jerk"][0], row["errors"]["mixed_sp"]["jerk"][0],
                row["sweep_ms"]["fp64"], row["sweep_ms"]["mixed"], row["sweep_ms"]["mixed_sp"]))
    return {"config": "precision_vs_n_plummer", "error_stats": "median, p99, max", "rows": rows}


def e2(ctx, t_end=0.125, n=262144, seed=6):
    """Block runs with FP64 (mixed) and FP32 (mixed_sp) jerk sums side by
    side: the paper finds no difference in energy conservation (Section 4).
    Both sweep every block with FP32 pair arithmetic."""
    x, v, m = inputs.plummer(n, seed)
    eps2 = (4.0 / n) ** 2
    p = _params(0.02)
    out = {"config": "plummer_n%d_jerk_sum_precision" % n, "t_end": t_end, "runs": {}}
    with _fp32_mixed(ctx):
        for pname in ("mixed", "mixed_sp"):
            s = H.State(x, v, m, TB)
            ctx.initialize(s, eps2, p, H.PRECISIONS[pname])
            out["runs"][pname] = block_run(ctx, s, eps2, p, t_end, H.PRECISIONS[pname],
                                           label="e2 " + pname)
    return out


def e4(ctx, t_end=1.0, ns=(1024, 2048, 4096, 8192, 16384), seed=7, form="paper"):
    """Whole-run interactions/s and GFLOPS (60 flops per interaction)
    against N, from t = 0 to t_end (Section 5, Fig. of GFLOPS vs N); eta =
    0.02 in the printed form eta sqrt(R) or the classic sqrt(eta R)."""
    rows = []
    p = _params(0.02, FORMS[form])
    for n in ns:
        x, v, m = inputs.plummer(n, seed)
        eps2 = (4.0 / n) ** 2
        for pname in ("fp64", "mixed"):
            s = H.State(x, v, m, TB)
            ctx.initialize(s, eps2, p, H.PRECISIONS[pname])
            r = block_run(ctx, s, eps2, p, t_end, H.PRECISIONS[pname],
                          label="e4 n%d %s" % (n, pname))
            r.update({"n": n, "precision": pname})
            rows.append(r)
    return {"config": "plummer_speed_vs_n", "t_end": t_end, "dt_form": form, "rows": rows}


def o1(ctx, ns=(1 << 20, 1 << 22, 1 << 24), reps=20, seed=8):
    """Achieved HBM bandwidth of the O(N) stages, against the 8 TB/s peak.
    The state is synthetic (uniform positions and velocities, small a and j,
    t = 0, every dt = 2^-10): the stages' cost does not depend on the
    physics.  Bytes per particle, counted from the kernels' loads and stores:
    select 3 x 16 B read (t, dt in the minimum, count and write passes) +
    4 B written (idx); predict 104 B read (x, v, a, j, t) + 48 B written
    (xp, vp); correct (every particle active) 164 B read (idx, dt, xp, vp,
    a, j and the new acc, jerk, pot) + 120 B written (x, v, a, j, pot, t,
    dt)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    rows = []
    for n in ns:
        f64 = dict(dtype=torch.float64, device="cuda")
        s = H.State(torch.zeros(3, n, **f64), torch.zeros(3, n, **f64),
                    torch.full((n,), 1.0 / n, **f64), TB)
        for t_ in (s.x, s.v):
            t_.uniform_(-1.0, 1.0, generator=g)
        for t_ in (s.a, s.j):
            t_.uniform_(-1e-3, 1e-3, generator=g)
        s.dt.fill_(1 << (TB - 10))
        idx = torch.empty(n, dtype=torch.int32, device="cuda")
        na = torch.empty(1, dtype=torch.int32, device="cuda")
        T = torch.empty(1, dtype=torch.int64, device="cuda")
        acc = s.a.clone()
        jrk = s.j.clone()
        pot = torch.zeros(n, **f64)
        p = _params(0.02)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps * 1e-3

        t_sel = timed(lambda: ctx.select_block(s, idx, na, T))
        t_pred = timed(lambda: ctx.predict(s, T_host=1 << (TB - 10)))

        def corr():
            # every particle active at T = dt (the state is reset each time)
            s.t.zero_()
            s.dt.fill_(1 << (TB - 10))
            ctx.correct(s, idx, acc, jrk, pot, p, T_host=1 << (TB - 10), n_act_max=n)
        t_fill = timed(lambda: (s.t.zero_(), s.dt.fill_(1 << (TB - 10))))
        t_corr = timed(corr) - t_fill
        row = {"n": n}
        for name, sec, byt in (("select", t_sel, 52), ("predict", t_pred, 152),
                               ("correct", t_corr, 284)):
            row[name] = {"us": sec * 1e6, "bytes_per_particle": byt,
                         "GB_per_s": byt * n / sec / 1e9,
                         "frac_of_8TBps": byt * n / sec / 8e12}
        rows.append(row)
        _log("  o1 N %9d  select %.0f GB/s  predict %.0f GB/s  correct %.0f GB/s"
             % (n, row["select"]["GB_per_s"], row["predict"]["GB_per_s"],
                row["correct"]["GB_per_s"]))
        del s, idx, acc, jrk, pot
        torch.cuda.empty_cache()
    return {"config": "o_n_stages_bandwidth", "rows": rows}


RUNNERS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "e1": e1, "e2": e2, "e3": e3,
           "e4": e4, "o1": o1}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(RUNNERS))
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--serial-t-end", type=float, default=None)
    ap.add_argument("--serial-clusters", type=int, default=None)
    ap.add_argument("--form", choices=sorted(FORMS), default=None,
                    help="timestep criterion form (default: as printed)")
    ap.add_argument("--start-div", type=float, default=0.0,
                    help="start-up factor = steady factor / this (0: the steady factor)")
    ap.add_argument("--tick-bits", type=int, default=None,
                    help="time tick 2^-tick_bits (default 20)")
    ap.add_argument("--k-min", type=int, default=None,
                    help="coarsest step 2^-k_min (default 3; a run ends on its multiple)")
    ap.add_argument("--k-max", type=int, default=None,
                    help="finest step 2^-k_max (default 20; at most tick_bits)")
    ap.add_argument("--max-wall", type=float, default=0.0,
                    help="stop a block run after this many seconds (0: run to the end)")
    ap.add_argument("--precision", choices=sorted(H.PRECISIONS), default=None,
                    help="c3, c4, c5: run in this precision instead of the configured one")
    ap.add_argument("--fp64-below", type=int, default=None,
                    help="mixed precisions: sweep systems below this size in FP64 "
                         "(library default 32768; 0: every system in FP32)")
    ap.add_argument("--etas", default=None,
                    help="e3: comma-separated eta values (default 0.0025 .. 0.08)")
    ap.add_argument("--small-blocks", type=int, default=None,
                    help="mixed precisions: blocks below this many interactions are swept "
                         "in FP64 (library default 5e7; 0: never)")
    ap.add_argument("--tune-cache", default=None,
                    help="c3: autotune every point of the latency curve into this cache")
    ap.add_argument("--no-run", action="store_true", help="c3: the latency curve only")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    global START_DIV, TB, K_MIN, K_MAX, MAX_WALL, RUN_FORM
    START_DIV = a.start_div
    MAX_WALL = a.max_wall
    if a.tick_bits is not None:
        TB = a.tick_bits
    if a.k_max is not None:
        K_MAX = a.k_max
    if a.k_min is not None:
        K_MIN = a.k_min
    ctx = H.Context(0)
    if a.precision is not None:
        RUN_PREC["p"] = H.PRECISIONS[a.precision]
    if a.small_blocks is not None:
        for prec in (H.MIXED, H.MIXED_2F):
            ctx.set_mixed_small_blocks(prec, a.small_blocks)
    if a.fp64_below is not None:
        for prec in (H.MIXED, H.MIXED_2F):
            near, _ = ctx.get_mixed_policy(prec)
            ctx.set_mixed_policy(prec, near, a.fp64_below)
    kw = {}
    if a.t_end is not None:
        kw["t_end"] = a.t_end
    if a.name == "c3" and a.tune_cache:
        kw["tune_cache"] = a.tune_cache
    if a.name == "c3" and a.no_run:
        kw["run"] = False
    if a.name == "c4" and a.serial_t_end is not None:
        kw["serial_t_end"] = a.serial_t_end
    if a.name == "c4" and a.serial_clusters is not None:
        kw["serial_clusters"] = a.serial_clusters
    if a.name == "e3" and a.etas:
        kw["etas"] = tuple(float(e) for e in a.etas.split(","))
    if a.name in ("e3", "e4") and a.form is not None:
        kw["form"] = a.form
    elif a.form is not None:
        RUN_FORM = FORMS[a.form]
    _log("workload %s %s" % (a.name, kw))
    res = RUNNERS[a.name](ctx, **kw)
    res["device"] = torch.cuda.get_device_name(0)
    res["start_div"] = START_DIV
    res["tick_bits"] = TB
    res["criterion_form"] = "paper" if RUN_FORM == H.DT_PAPER else "aarseth"
    res["mixed_policy"] = list(ctx.get_mixed_policy(H.MIXED)) + [
        ctx.get_mixed_small_blocks(H.MIXED)]
    res["precision_override"] = a.precision
    res["k_min_max"] = [K_MIN, K_MAX]
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
