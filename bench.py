"""Benchmark: the Hermite block step of a Plummer sphere, N = 65536, on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

One timed step is one pass of the whole hot path over the system: block
selection, prediction of all particles, the force/jerk/potential sweep of
the active block, and the corrector with the next Aarseth step.  Before each
step every particle's step size is reset to one shared step h = 2^-12, so
the active block is all N particles and every step does N^2 interactions
(the paper's full-N workload; Section 5).  Positions keep advancing.

Metric: interactions/s (N_act * N per step) and GFLOPS at the paper's 60
flops per interaction, for the mixed path (headline) and the FP64 path.
The mixed path runs with the library's default policy: FP64 near field and
the FP64 refinement of the particles whose FP32 rounding estimate exceeds
the bound, so that every particle meets 1e-6 (the count refined per step is
reported).  The roofline entry is for the sweep kernel (the dominant
kernel), with its average duration measured by HIP events recorded on the
launch stream around the sweep launches alone (the mixed sweep is launched
with its FP64 half, which leaves at once for a full-N block and takes a few
microseconds), priced at 42 algorithmic flops per
interaction (count of the operations in the force, jerk and potential
equations, FMA = 2); the whole force call (plan, sweep, reduce/refine) is
reported beside it.  Both FP32 difference forms of the mixed sweep (cast and
split hi/lo) are timed and checked.  The cpu_baseline entry times the FP64
CPU oracle on a bounded sample of active particles of the same state.  The
batched entry sweeps the 256-cluster ensemble with every particle active in
one launch, FP64 against mixed, as a fraction of the vector peaks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 65536
SEED = 3
ETA = 0.02
TB = 20
H_SHARED_K = 12                      # shared step 2^-12 for the timed steps
FLOPS_PAPER = 60                     # per interaction, the paper's convention
FLOPS_ALGO = 42                      # per interaction, operation count
PEAK_FP64 = 78.6e12                  # MI355X vector FP64, FLOP/s
PEAK_FP32 = 157.3e12                 # MI355X vector FP32 (packed), FLOP/s
PEAK_FP32_UNPACKED = 78.6e12         # FP32 as issued by this build
# The paper's own throughput, quoted as context with its hardware (Section 5,
# Table 4, Turbo Boost on: AVX on an Intel Core i7-2600 at N = 16K, the
# largest N it measures; it has no figure at N = 64K).
PAPER_FIGURES = {
    "hardware": "Intel Core i7-2600 (Sandy Bridge, 4 cores, 3.4 GHz), AVX, CPU",
    "n": 16384,
    "gflops_60_1core_1proc": 20.5,
    "gflops_60_4cores_8procs": 90.9,
    "interactions_per_s_4cores_8procs": 90.9e9 / FLOPS_PAPER,
    "source": "Section 5, Table 4, Turbo Boost on",
}
METRIC = ("force+jerk interactions/s & GFLOPS (N=65536); mixed vs FP64 at "
          "≤1e-6 rel err")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other FP32 difference form of the mixed sweep")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape")
    ap.add_argument("--tuning-cache", default=os.path.join(tempfile.gettempdir(),
                                                           "hermite_tuning.json"),
                    help="autotuner cache: loaded if it has this size, else written")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even when the committed counter summary names a shape")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-cluster ensemble sweep (it runs only when "
                         "--precisions holds both fp64 and mixed)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on one GPU (the sweep "
              "would shard over GPUs by splitting the j range, each GPU summing its "
              "share for every active particle); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calib:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": 256 << 20, "reps": 5}))
        return
    from paper_1104_2700_amd import hermite as H, inputs

    x, v, m = inputs.plummer(N, SEED)
    eps2 = (4.0 / N) ** 2
    ctx = H.Context(0)
    params = H.dt_params(ETA, H.DT_PAPER, 3, 20)
    base = H.State(x, v, m, TB)
    ctx.initialize(base, eps2, params, H.FP64)
    torch.cuda.synchronize()
    h_ticks = 1 << (TB - H_SHARED_K)

    results = {}
    precs = [p for p in args.precisions.split(",") if p]
    prof = None if args.retune else profiled_counters(None)
    for pname in precs:
        prec = H.PRECISIONS[pname]
        shape = prof.get(pname, {}).get("tuning") if prof else None
        if shape and not args.no_autotune:
            # the (autotuned) launch shape the committed counters were taken at,
            # while the sweep's sources are unchanged
            t = ctx.get_tuning(prec)
            for k, val in shape.items():
                setattr(t, k, int(val))
            ctx.set_tuning(prec, t)
        elif not args.no_autotune and not ctx.load_tuning(args.tuning_cache, prec, N, N):
            # pick the sweep's launch shape for this size (untimed set-up)
            ts = base.clone()
            ts.xp.copy_(ts.x)
            ts.vp.copy_(ts.v)
            ctx.autotune(ts, eps2, prec, N, cache_path=args.tuning_cache)
            del ts
        tuning = ctx.get_tuning(prec).as_dict()
        s = base.clone()
        s.dt.fill_(h_ticks)

        def one_step():
            s.dt.fill_(h_ticks)
            ctx.step(s, eps2, params, prec, use_graph=not args.no_graph)

        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        c0 = ctx.counters()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cnt = ctx.counters()
        assert cnt["n_act"] == N, cnt
        ms_step = 1e3 * wall / args.steps
        inter_s = N * N / (wall / args.steps)
        refined = (cnt["refined"] - c0["refined"]) / args.steps
        # kernel-level timing of the force call at the same launch shape: HIP
        # events on the launch stream around the plan kernel, the sweep
        # kernel and the finishing kernels (reduce; flag, FP64 refine sweep
        # and scatter for the refining mixed sweep)
        fs = base.clone()
        fs.xp.copy_(fs.x)
        fs.vp.copy_(fs.v)
        reps = max(10, args.steps)
        acc, jrk, pot, _ = ctx.force_jerk_timed(fs, None, eps2, prec, reps=2)
        acc, jrk, pot, ph = ctx.force_jerk_timed(fs, None, eps2, prec, reps=reps,
                                                 acc=acc, jerk=jrk, pot=pot)
        results[pname] = {
            "ms_per_step": ms_step, "interactions_per_s": inter_s,
            "gflops_60": inter_s * FLOPS_PAPER / 1e9,
            "refined_per_step": refined,
            "force_ms": ph,
            "sweep_kernel_interactions_per_s": N * N / (ph["sweep"] * 1e-3),
            "force_call_interactions_per_s": N * N / (ph["total"] * 1e-3),
            "tuning": tuning,
            "out": (acc.cpu().numpy(), jrk.cpu().numpy(), pot.cpu().numpy()),
        }
        if pname in ("mixed", "mixed2f") and not args.no_variants:
            # the other form of the FP32 differences (cast <-> split hi/lo),
            # same launch shape otherwise
            t = ctx.get_tuning(prec)
            keep = t.variant
            t.variant = keep ^ 2
            ctx.set_tuning(prec, t)
            a2, j2, p2, ph2 = ctx.force_jerk_timed(fs, None, eps2, prec, reps=reps)
            t.variant = keep
            ctx.set_tuning(prec, t)
            form = "split" if (keep ^ 2) & 2 else "cast"
            results[pname + "_" + form] = {
                "force_ms": ph2, "tuning": dict(tuning, variant=keep ^ 2),
                "sweep_kernel_interactions_per_s": N * N / (ph2["sweep"] * 1e-3),
                "force_call_interactions_per_s": N * N / (ph2["total"] * 1e-3),
                "out": (a2.cpu().numpy(), j2.cpu().numpy(), p2.cpu().numpy()),
            }
        del fs

    # every particle of the mixed outputs against the FP64 sweep of the
    # same state (the FP64 path is held to the oracle at 1e-13 by the tests)
    if "fp64" in results:
        A0, J0, P0 = results["fp64"]["out"]
        for p, r in results.items():
            if p == "fp64":
                continue
            A, J, P = r["out"]
            ea = np.linalg.norm(A - A0, axis=0) / np.linalg.norm(A0, axis=0)
            ej = np.linalg.norm(J - J0, axis=0) / np.linalg.norm(J0, axis=0)
            ep = np.abs(P - P0) / np.abs(P0)
            r["all_particles_vs_fp64_sweep"] = {
                "acc_rel_max": float(ea.max()), "jerk_rel_max": float(ej.max()),
                "jerk_rel_p999": float(np.percentile(ej, 99.9)),
                "jerk_n_above_1e-6": int((ej > 1e-6).sum()),
                "acc_n_above_1e-6": int((ea > 1e-6).sum()),
                "pot_rel_max": float(ep.max())}

    batched = None
    if not args.no_batched and "fp64" in results and "mixed" in results:
        batched = batched_leg(ctx, H, inputs, max(10, args.steps), not args.no_autotune)

    cpu = None
    accuracy = {}
    if not args.no_cpu:
        cpu, accuracy = cpu_leg(x, v, m, eps2, results, args.cpu_seconds)

    head = "mixed" if "mixed" in results else precs[0]
    r = results[head]
    sweep_ms = r["force_ms"]["sweep"]
    achieved = FLOPS_ALGO * N * N / (sweep_ms * 1e-3)
    peak = PEAK_FP32 if head != "fp64" else PEAK_FP64
    prof = profiled_counters()
    traffic = issued = None
    # counters hold for the launch shape they were taken at (the j-split sets
    # the partial-sum traffic)
    if prof is not None and head in prof and prof[head].get("tuning") == r["tuning"]:
        traffic = prof[head]["traffic_bytes"]
        fl = prof[head]["fp32_flops_per_interaction"] + prof[head]["fp64_flops_per_interaction"]
        issued = fl * N * N / (sweep_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": r["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32 mixed" if head != "fp64" else "f64",
        "data": "synthetic Plummer sphere (Henon units), N=65536, seed 3",
        "config": {"workload": "plummer_n65536_full_block_step", "n": N, "n_act": N,
                   "eps": 4.0 / N, "eta": ETA, "precision": head,
                   "shared_step": 2.0 ** -H_SHARED_K,
                   "graph": not args.no_graph},
        "gflops_60": r["gflops_60"],
        "paths": {p: {k: v for k, v in q.items() if k != "out"} for p, q in results.items()},
        "accuracy_vs_oracle": accuracy,
        "roofline": {
            "bound": "alu",
            "kernel": "force sweep kernel (hermite_sweep), precision %s, variant %d"
                      % (head, r["tuning"]["variant"]),
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "issued_tflops_from_counters": issued,
            "flops_per_interaction": FLOPS_ALGO,
            "kernel_ms": sweep_ms,
            "force_call_ms": r["force_ms"]["total"],
            "force_call_frac": FLOPS_ALGO * N * N / (r["force_ms"]["total"] * 1e-3) / peak,
            "frac_vs_fp64_or_unpacked_fp32_peak": achieved / PEAK_FP64,
        },
        "cpu_baseline": cpu,
        "paper_figures": PAPER_FIGURES,
    }
    if batched is not None:
        out["batched"] = batched
    if "fp64" in results and head != "fp64":
        f = results["fp64"]
        out["fp64_vs_mixed"] = {
            "fp64_interactions_per_s": f["interactions_per_s"],
            "mixed_speedup_step": r["interactions_per_s"] / f["interactions_per_s"],
            "mixed_speedup_force_call": f["force_ms"]["total"] / r["force_ms"]["total"],
            "fp64_sweep_frac_fp64_peak":
                FLOPS_ALGO * N * N / (f["force_ms"]["sweep"] * 1e-3) / PEAK_FP64,
        }
    print(json.dumps(out), flush=True)


def batched_leg(ctx, H, inputs, reps, autotune):
    """The batched workload: the 256-cluster ensemble (N_c log-uniform in
    [256, 8192], eps_c = 4/N_c; 673 038 particles) with every particle
    active, swept in one persistent launch over all clusters (each cluster is
    its own system: Section 3.3's sweep per cluster, no pair across them).
    Timed in FP64 and in mixed precision twice: with the library's default
    policy, which sweeps systems below 32768 particles with the FP64 kernel,
    and with that rule off, so that every cluster is swept in FP32 (near
    field and refinement kept).  The launch shapes are autotuned for this
    workload (untimed); HIP events on the launch stream time the sweep
    kernels and the whole force call, averaged over ``reps`` calls."""
    import torch
    x, v, m, off, eps = inputs.ensemble()
    n = int(off[-1])
    cl = H.Clusters(off, eps ** 2)
    s = H.State(x, v, m, TB)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    sizes = np.diff(off).astype(np.float64)
    inter = float((sizes * sizes).sum())
    near, below = ctx.get_mixed_policy(H.MIXED)
    rows = (("fp64", H.FP64, below), ("mixed_default_policy", H.MIXED, below),
            ("mixed_fp32_sweeps", H.MIXED, 0))
    if autotune:
        ctx.autotune(s, 0.0, H.FP64, n, clusters=cl)
        ctx.set_mixed_policy(H.MIXED, near, 0)
        ctx.autotune(s, 0.0, H.MIXED, n, clusters=cl)
    out = {"workload": "ensemble_256_clusters_n256_8192_all_active",
           "n_clusters": int(off.shape[0] - 1), "n_particles": n,
           "interactions_per_sweep": inter}
    ref = None
    for label, prec, fp64_below in rows:
        ctx.set_mixed_policy(H.MIXED, near, fp64_below)
        a, j, p, _ = ctx.force_jerk_timed(s, None, 0.0, prec, reps=2, clusters=cl)
        a, j, p, ph = ctx.force_jerk_timed(s, None, 0.0, prec, reps=reps, acc=a, jerk=j,
                                           pot=p, clusters=cl)
        torch.cuda.synchronize()
        peak = PEAK_FP64 if label != "mixed_fp32_sweeps" else PEAK_FP32
        row = {"force_call_interactions_per_s": inter / (ph["total"] * 1e-3),
               "sweep_kernel_interactions_per_s": inter / (ph["sweep"] * 1e-3),
               "gflops_60": FLOPS_PAPER * inter / (ph["total"] * 1e-3) / 1e9,
               "sweep_frac_of_peak": FLOPS_ALGO * inter / (ph["sweep"] * 1e-3) / peak,
               "peak": "fp64" if peak == PEAK_FP64 else "fp32",
               "force_ms": ph, "tuning": ctx.get_tuning(prec).as_dict()}
        A, J, P = a.cpu().numpy(), j.cpu().numpy(), p.cpu().numpy()
        if ref is None:
            ref = (A, J, P)
        else:
            A0, J0, _ = ref
            ea = np.linalg.norm(A - A0, axis=0) / np.linalg.norm(A0, axis=0)
            ej = np.linalg.norm(J - J0, axis=0) / np.linalg.norm(J0, axis=0)
            row["vs_fp64_sweep"] = {"acc_rel_max": float(ea.max()),
                                    "jerk_rel_max": float(ej.max()),
                                    "acc_n_above_1e-6": int((ea > 1e-6).sum()),
                                    "jerk_n_above_1e-6": int((ej > 1e-6).sum())}
        out[label] = row
    ctx.set_mixed_policy(H.MIXED, near, below)
    return out


def profiled_counters(_unused=None):
    """Per-launch HBM traffic and issued FLOPs of the sweep from the committed
    rocprofv3 counter summary, if the sweep's sources are unchanged since it
    was taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sweep_n65536_traffic.json")
    try:
        with open(path) as f:
            prof = json.load(f)
        src = b""
        for name in ("sweep.hip", "plan.h"):
            with open(os.path.join(ROOT, "paper_1104_2700_amd", "csrc", name), "rb") as f:
                src += f.read()
        if hashlib.sha256(src).hexdigest() != prof.get("source_sha256"):
            return None
        return prof
    except (OSError, ValueError):
        return None


def cpu_leg(x, v, m, eps2, results, target_s):
    """Times the FP64 oracle on a sample of active particles of the same
    state, on every host core it is given, and measures the GPU outputs'
    error against it on the 1024-particle evaluation sample."""
    from oracle import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    eval_idx = np.sort(np.random.default_rng(1003).choice(N, 1024, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    ra, rj, rp = O.force(x, v, m, eval_idx, eps2)
    t1 = time.perf_counter()
    rate0 = 1024 * N / (t1 - t0)
    extra = int(min(N - 1024, max(0, rate0 * target_s / N - 1024)))
    rng = np.random.default_rng(7)
    rest = np.setdiff1d(np.arange(N, dtype=np.int32), eval_idx)
    more = np.sort(rng.choice(rest, size=extra, replace=False)).astype(np.int32)
    t2 = time.perf_counter()
    if extra:
        O.force(x, v, m, more, eps2)
    t3 = time.perf_counter()
    n_i = 1024 + extra
    secs = (t1 - t0) + (t3 - t2)
    cpu = {"value": n_i * N / secs, "unit": "interactions/s", "cores": cores,
           "kind": "oracle",
           "sample": "%d active particles x %d j of the N=65536 Plummer state "
                     "(FP64, Neumaier sums), %.1f s" % (n_i, N, secs)}
    # the same sweep on one host thread, on a smaller sample
    prev = O.threads()
    O.threads(1)
    one_idx = eval_idx[:256]
    t4 = time.perf_counter()
    O.force(x, v, m, one_idx, eps2)
    t5 = time.perf_counter()
    O.threads(prev)
    cpu["single_thread"] = {"value": one_idx.shape[0] * N / (t5 - t4), "unit": "interactions/s",
                            "cores": 1, "sample": "256 active particles x %d j" % N}
    # the whole N = 1024 run (Plummer seed 1, eps = 1/64, eta = 0.02, t = 0 -> 0.125)
    from paper_1104_2700_amd import inputs
    x1, v1, m1 = inputs.plummer(1024, 1)
    st = O.new_state(x1, v1, m1, TB)
    t6 = time.perf_counter()
    stats = O.run(st, 1 << (TB - 3), (1.0 / 64) ** 2, ETA, O.FORM_PAPER, 3, 20)
    t7 = time.perf_counter()
    cpu["n1024_run"] = {"value": stats["interactions"] / (t7 - t6), "unit": "interactions/s",
                        "cores": cores, "wall_s": t7 - t6, "block_steps": stats["steps"],
                        "gflops_60": FLOPS_PAPER * stats["interactions"] / (t7 - t6) / 1e9}
    acc = {}
    for p, r in results.items():
        A, J, P = r["out"]
        ea = np.linalg.norm(A[:, eval_idx] - ra, axis=0) / np.linalg.norm(ra, axis=0)
        ej = np.linalg.norm(J[:, eval_idx] - rj, axis=0) / np.linalg.norm(rj, axis=0)
        ep = np.abs(P[eval_idx] - rp) / np.abs(rp)
        acc[p] = {"sample": 1024,
                  "acc_rel_median": float(np.median(ea)), "acc_rel_max": float(ea.max()),
                  "jerk_rel_median": float(np.median(ej)), "jerk_rel_p99": float(np.percentile(ej, 99)),
                  "jerk_rel_max": float(ej.max()), "jerk_n_above_1e-6": int((ej > 1e-6).sum()),
                  "pot_rel_median": float(np.median(ep)), "pot_rel_max": float(ep.max())}
    return cpu, acc


if __name__ == "__main__":
    main()
