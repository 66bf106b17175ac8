"""Whole-run workloads on one GPU (block-timestep integrations).

    python -m paper_1104_2700_amd.workloads <name> [--t-end T] [--out file.json]

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

Every run reports wall time, block steps, interactions, interactions/s,
GFLOPS at the paper's 60 flops per interaction (Section 5), clamped steps
and the relative energy change (energies from FP64 potential sweeps at the
synchronised start and end, Section 4).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import hermite as H
from . import inputs

TB = 20          # time tick 2^-20
K_MIN, K_MAX = 3, 20


def _log(msg):
    print(msg, flush=True)


def _energy(ctx, s, eps2, clusters=None):
    e = ctx.energy(s, eps2, clusters=clusters).cpu().numpy()
    return e[:, 0] + e[:, 1]


def block_run(ctx, s, eps2, params, t_end, precision, clusters=None,
              chunk=20000, label=""):
    """Integrates an initialised state to t_end (time units), printing a
    progress line every `chunk` launched steps.  Returns a dict of stats."""
    T_end = int(round(t_end * (1 << TB)))
    e0 = _energy(ctx, s, eps2, clusters)
    c0 = ctx.counters()
    h0 = np.array(ctx.block_histogram())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = inter = 0
    while True:
        st, it, done = ctx.run(s, eps2, params, T_end, precision, use_graph=True,
                               sync_every=256, clusters=clusters, max_steps=chunk,
                               with_done=True)
        steps += st
        inter += it
        cnt = ctx.counters()
        _log("  %s t = %.6f  block steps %d  interactions %.3e  %.1f s"
             % (label, cnt["T"] / (1 << TB), steps, inter, time.perf_counter() - t0))
        if done:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e1 = _energy(ctx, s, eps2, clusters)
    c1 = ctx.counters()
    hist = (np.array(ctx.block_histogram()) - h0).tolist()
    rel = np.abs((e1 - e0) / e0)
    return {
        "t_end": t_end, "wall_s": wall, "block_steps": steps, "interactions": inter,
        "interactions_per_s": inter / wall, "gflops_60": 60.0 * inter / wall / 1e9,
        "clamped_steps": c1["clamped"] - c0["clamped"],
        "energy_rel_change_max": float(rel.max()),
        "energy_rel_change_median": float(np.median(rel)),
        "E0": float(e0.sum()) if e0.size == 1 else None,
        "active_size_histogram_log2": {("0" if b == 0 else "[2^%d,2^%d)" % (b - 1, b)): v
                                       for b, v in enumerate(hist) if v},
        "mean_active": inter / max(steps, 1) / (s.n if clusters is None else 1),
    }


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
    p = H.dt_params(0.02, H.DT_PAPER, K_MIN, K_MAX)
    ctx.initialize(s, eps2, p, H.FP64)
    return {"config": "plummer_n1024_fp64", "run": block_run(ctx, s, eps2, p, t_end, H.FP64,
                                                             label="c1")}


def c2(ctx, t_end=1.0):
    n = 16384
    s = _plummer_state(n, 2)
    eps2 = (4.0 / n) ** 2
    p = H.dt_params(0.02, H.DT_PAPER, K_MIN, K_MAX)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    ms = sweep_time(ctx, s, eps2, H.FP64)
    ctx.initialize(s, eps2, p, H.FP64)
    run = block_run(ctx, s, eps2, p, t_end, H.FP64, label="c2")
    return {"config": "plummer_n16384_fp64",
            "full_sweep": {"ms": ms, "interactions_per_s": n * n / (ms * 1e-3),
                           "gflops_60": 60 * n * n / (ms * 1e-3) / 1e9},
            "run": run}


def c3(ctx, t_end=1.0):
    n = 65536
    s = _plummer_state(n, 3)
    eps2 = (4.0 / n) ** 2
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    curve = []
    na = 1
    while na <= n:
        idx = torch.arange(0, n, n // na, dtype=torch.int32, device="cuda")[:na].contiguous()
        row = {"n_act": na}
        for pname in ("fp64", "mixed"):
            ms = sweep_time(ctx, s, eps2, H.PRECISIONS[pname], idx, reps=20)
            row[pname + "_us"] = 1e3 * ms
            row[pname + "_interactions_per_s"] = na * n / (ms * 1e-3)
        curve.append(row)
        _log("  c3 n_act %6d  fp64 %.1f us  mixed %.1f us" % (na, row["fp64_us"], row["mixed_us"]))
        na *= 2
    p = H.dt_params(0.02, H.DT_PAPER, K_MIN, K_MAX)
    ctx.initialize(s, eps2, p, H.MIXED)
    run = block_run(ctx, s, eps2, p, t_end, H.MIXED, label="c3")
    return {"config": "plummer_n65536_mixed", "latency_curve": curve, "run": run}


def c4(ctx, t_end=0.5, serial_t_end=0.125, n_clusters=256, serial_clusters=16):
    """Batched ensemble run, then batched vs serial on a subset of clusters."""
    x, v, m, off, eps = inputs.ensemble(n_clusters, 4)
    eps2 = eps ** 2
    sizes = np.diff(off)
    p = H.dt_params(0.02, H.DT_PAPER, K_MIN, K_MAX)
    out = {"config": "ensemble_%d_clusters_mixed" % n_clusters,
           "n_total": int(off[-1]), "sum_Nc2": float(np.sum(sizes.astype(float) ** 2)),
           "sizes_min_max": [int(sizes.min()), int(sizes.max())]}
    cl = H.Clusters(off, eps2)
    s = H.State(x, v, m, TB)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    out["tuning"] = ctx.autotune(s, 0.0, H.MIXED, int(off[-1]), clusters=cl).as_dict()
    ctx.initialize(s, 0.0, p, H.MIXED, clusters=cl)
    out["batched"] = block_run(ctx, s, 0.0, p, t_end, H.MIXED, clusters=cl, label="c4 batched")
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
    p = H.dt_params(0.02, H.DT_PAPER, K_MIN, K_MAX)
    ctx.initialize(s, eps2, p, H.MIXED_2F)
    return {"config": "plummer_imf_binaries_n131072_mixed2f",
            "run": block_run(ctx, s, eps2, p, t_end, H.MIXED_2F, label="c5")}


RUNNERS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(RUNNERS))
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--serial-t-end", type=float, default=None)
    ap.add_argument("--serial-clusters", type=int, default=None)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    ctx = H.Context(0)
    kw = {}
    if a.t_end is not None:
        kw["t_end"] = a.t_end
    if a.name == "c4" and a.serial_t_end is not None:
        kw["serial_t_end"] = a.serial_t_end
    if a.name == "c4" and a.serial_clusters is not None:
        kw["serial_clusters"] = a.serial_clusters
    _log("workload %s %s" % (a.name, kw))
    res = RUNNERS[a.name](ctx, **kw)
    res["device"] = torch.cuda.get_device_name(0)
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
