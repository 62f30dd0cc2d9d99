#!/usr/bin/env python3
"""Fill-throughput benchmark of the gfx950 histogram library on one GPU.

Workload (default): the variable-bin 1D fill -- 99,999 log-spaced bins (1e5
edges on [1e-3, 1e3]), 5e7 events x ~ Exp(1) in binary64, unit weights, seed
1 -- with the learned find-bin index (binary search is timed beside it).  One
step is one hist_fill of all 5e7 events: find bin, LDS accumulation, merge and
the statistics sums, with the inputs already resident in HBM.

Prints one JSON line (rank 0).  Fields beyond the driver contract:
  roofline      HBM roofline of the dominant kernel (the fill kernel), with
                its duration measured by HIP events on its launch stream
  cpu_baseline  the CPU oracle timed on the host on one full step of the same
                workload (single thread)
  bsearch       the same fill with plain binary search on the variable axis
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fill events/s + HBM GB/s fraction; learned vs bsearch FindBin, 1 GPU"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="variable_1d",
                    choices=["variable_1d", "plain_1d", "corr_3d", "precision", "paper_1d"])
    ap.add_argument("--events", type=int, default=0, help="override the event count")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-bsearch", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM traffic per launch measured with rocprofv3 counters")
    return ap.parse_args()


def build_workload(name, events):
    import synth
    if name == "variable_1d":
        return synth.variable_1d(events or synth.VARIABLE_1D_N)
    if name == "plain_1d":
        return synth.plain_1d(events or synth.PLAIN_1D_N)
    if name == "corr_3d":
        return synth.corr_3d(events or synth.CORR_3D_N)
    if name == "paper_1d":
        return synth.paper_1d(events or 500_000_000 // 10)
    if name == "precision":
        import numpy as np
        n = events or synth.PRECISION_SLICE
        x, w = next(synth.precision_slices(n=n, slice_len=n))
        return {"name": "precision", "axes": synth.precision_axes(), "coords": [x], "weights": w}
    raise ValueError(name)


def describe(wl, n):
    ax = wl["axes"]
    parts = []
    for a in ax:
        if a.get("edges") is not None:
            parts.append("%d variable bins [%g, %g]" % (a["nbins"], a["edges"][0], a["edges"][-1]))
        else:
            parts.append("%d fixed bins [%g, %g)" % (a["nbins"], a["xmin"], a["xmax"]))
    w = "unit weights" if wl["weights"] is None else "weights"
    dt = str(wl["coords"][0].dtype)
    return "%s: %s; %d events, %s, %s" % (wl["name"], " x ".join(parts), n, dt, w)


def alg_bytes(wl, n):
    """Algorithmic HBM bytes of one fill: every coordinate and weight read
    once, the final sums of weights and squared weights written once (FP64),
    each edge array read once."""
    esz = wl["coords"][0].dtype.itemsize
    per_event = len(wl["coords"]) * esz + (0 if wl["weights"] is None else esz)
    T = 1
    edges = 0
    for a in wl["axes"]:
        T *= a["nbins"] + 2
        if a.get("edges") is not None:
            edges += (a["nbins"] + 1) * 8
    return per_event * n + 16 * T + edges, per_event


def time_fills(hg, h, cols, w, steps, warmup):
    import torch
    for _ in range(warmup):
        h.fill(cols, w)
    torch.cuda.synchronize()
    h.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.fill(cols, w)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = h.timing_read()
    h.timing(False)
    return wall, kt


def cpu_baseline(wl, n):
    import oracle
    o = oracle.Oracle(wl["axes"])
    cols = [c.astype("float64") for c in wl["coords"]]
    w = None if wl["weights"] is None else wl["weights"].astype("float64")
    t0 = time.perf_counter()
    o.fill(cols, w)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": "one full step (%d events, same arrays), sequential C oracle, %.2f s"
                      % (n, dt)}


def load_traffic(path, workload, n):
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(workload)
    if not rec or rec.get("events") != n:
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2401_13310_amd as hg

    torch.cuda.set_device(0)
    wl = build_workload(args.workload, args.events)
    n = wl["coords"][0].size
    cols = [torch.from_numpy(c).to("cuda") for c in wl["coords"]]
    w = None if wl["weights"] is None else torch.from_numpy(wl["weights"]).to("cuda")
    flags = hg.HIST_F_ACC_F32C if args.workload == "precision" else 0
    variable = any(a.get("edges") is not None for a in wl["axes"])

    h = hg.Hist(wl["axes"], flags)
    train_ms = None
    if variable:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, ax in enumerate(wl["axes"]):
            if ax.get("edges") is not None:
                h.train_index(a)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
    sample = min(n, 1 << 22)
    h.tune([c[:sample] for c in cols], None if w is None else w[:sample])
    plan = h.plan_info(n, hg.HIST_F32 if wl["coords"][0].dtype == np.float32 else hg.HIST_F64,
                       w is not None)

    wall, kt = time_fills(hg, h, cols, w, args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    value = n * args.steps / wall
    fill_ms = kt["fill_ms"] / max(1, kt["launches"])
    merge_ms = kt["merge_ms"] / max(1, kt["launches"])
    B, per_event = alg_bytes(wl, n)
    achieved = B / (fill_ms * 1e-3) / 1e9
    traffic = load_traffic(args.traffic, args.workload, n)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["coords"][0].dtype == np.float32 else "f64",
        "data": "synthetic (seeded numpy PCG64), resident in HBM before timing",
        "config": {"workload": describe(wl, n),
                   "search": "learned" if variable else "fixed-width formula",
                   "plan": plan},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fill_kernel", "kernel_ms": fill_ms,
                     "merge_kernel_ms": merge_ms,
                     "alg_bytes_per_launch": B, "alg_bytes_per_event": per_event},
        "step_hbm_frac": B / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    if train_ms is not None:
        out["index_train_ms"] = train_ms
    if variable and not args.no_bsearch:
        hb = hg.Hist(wl["axes"], flags)
        hb.tune([c[:sample] for c in cols], None if w is None else w[:sample])
        wall_b, kt_b = time_fills(hg, hb, cols, w, max(3, args.steps // 2), 1)
        steps_b = max(3, args.steps // 2)
        out["bsearch"] = {"value": n * steps_b / wall_b, "ms_per_step": wall_b / steps_b * 1e3,
                          "kernel_ms": kt_b["fill_ms"] / max(1, kt_b["launches"]),
                          "plan": hb.plan_info(n, hg.HIST_F64, w is not None)}
        out["learned_speedup_vs_bsearch"] = out["value"] / out["bsearch"]["value"]
        hb.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, n)
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
