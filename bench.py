#!/usr/bin/env python3
"""Fill-throughput benchmark of the gfx950 histogram library on one GPU.

Headline workload (default): the variable-bin 1D fill -- 99,999 log-spaced
bins (1e5 edges on [1e-3, 1e3]), 5e7 events x ~ Exp(1) in binary64, unit
weights, seed 1 -- with the learned find-bin index (binary search is timed
beside it).  One step is one hist_fill of all 5e7 events: find bin, LDS
accumulation, merge and the statistics sums, with the inputs already resident
in HBM.

Prints one JSON line.  Fields beyond the driver contract:
  roofline      HBM roofline of the fill (every kernel of one hist_fill: the
                fill kernel plus its merge), durations from HIP events on the
                launch stream
  parity        the timed plan's result (one more fill after a reset) against
                the CPU oracle on the same arrays: counts bit-exact, statistics
                within 1e-12 of max(|value|, sum of |terms|)
  cpu_baseline  the CPU oracle timed on the host on one full step of the same
                workload (single thread), with an all-cores run beside it
  bsearch       the same fill with plain binary search on the variable axis
  configs       the other workloads (plain 1D, correlated 3D, 64 batched
                histograms, FP32 precision), each with throughput, roofline
                fraction and parity against the oracle; the FP32 workload also
                reports its per-bin and per-statistic error against binary64
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fill events/s + HBM GB/s fraction; learned vs bsearch FindBin, 1 GPU"
HBM_PEAK_GBS = 8000.0
REL = 1e-12
CONFIGS = ("C1", "C3", "C4", "C5", "F1", "F2")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="variable_1d",
                    choices=["variable_1d", "plain_1d", "corr_3d", "precision", "paper_1d",
                             "batched_64", "sweep"],
                    help="variable_1d (default) is the headline and also runs --configs; the "
                         "others time one workload on its own")
    ap.add_argument("--configs", default=",".join(CONFIGS),
                    help="comma-separated subset of %s run beside the headline ('' for none)"
                         % ",".join(CONFIGS))
    ap.add_argument("--events", type=int, default=0, help="override the event count")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle (baseline and parity)")
    ap.add_argument("--no-bsearch", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM traffic per launch measured with rocprofv3 counters")
    ap.add_argument("--ingest", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PLAN_JSON"),
                    help="read two rocprofv3 --pmc databases of a --profile run (FETCH_SIZE, "
                         "then WRITE_SIZE), scale each by the copy kernel of known size, and "
                         "record the HBM bytes per launch of the fill kernel and its merge kernel "
                         "in --traffic")
    ap.add_argument("--strategy", default="tuned", choices=["tuned", "lds", "global", "tiled", "part"],
                    help="profile runs: fix the accumulation strategy instead of tuning")
    ap.add_argument("--profile", action="store_true",
                    help="for counter runs: tune, run --steps fills, then 3 device copies of "
                         "the coordinate column (a copy of known size to scale the counters); "
                         "prints the plan, no JSON")
    return ap.parse_args()


FILL_SOURCES = ("fill.hip", "fill_learned.hip", "fill_shape.hip", "fill_body.h", "hist_internal.h",
                "device_common.h", "kernels.h")


def kernel_source_hash():
    """Hash of the sources the fill kernels compile from: counter-derived
    traffic is valid only for the kernels it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2401_13310_amd", "csrc")
    hs = hashlib.sha256()
    for name in FILL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            hs.update(name.encode() + b"\0" + f.read())
    return hs.hexdigest()[:16]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- host side --

def cpu_threads():
    """Host threads for the all-cores oracle: the process's CPUs, at most 16
    (the CPU share a one-GPU machine gives a process)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_fill(axes, coords, weights, threads):
    """The CPU oracle over the events, split into `threads` contiguous chunks
    filled concurrently (the oracle is C called through ctypes, which releases
    the interpreter lock) and summed in chunk order.  threads=1 is one plain
    sequential oracle fill.  Returns the histogram and the wall time."""
    import oracle
    n = len(coords[0])
    p = max(1, min(threads, n // 65536 if n >= 65536 else 1))
    bounds = [n * i // p for i in range(p + 1)]

    def work(i):
        b0, b1 = bounds[i], bounds[i + 1]
        o = oracle.Oracle(axes)
        o.fill([c[b0:b1] for c in coords], None if weights is None else weights[b0:b1])
        return o.read()

    t0 = time.perf_counter()
    if p == 1:
        parts = [work(0)]
    else:
        with ThreadPoolExecutor(p) as ex:
            parts = list(ex.map(work, range(p)))
    dt = time.perf_counter() - t0
    sumw = parts[0][0].copy()
    sumw2 = parts[0][1].copy()
    stats = parts[0][2].copy()
    entries = parts[0][3]
    for sw, sw2, st, en in parts[1:]:
        sumw += sw
        sumw2 += sw2
        stats += st
        entries += en
    return {"sumw": sumw, "sumw2": sumw2, "stats": stats, "entries": entries,
            "seconds": dt, "threads": p, "events": n}


def oracle_scale(axes, coords, weights, threads):
    """Sum of |per-event term| of every statistic (the tolerance scale of
    statistics that can cancel), over chunks in parallel."""
    import oracle
    n = len(coords[0])
    p = max(1, min(threads, n // 65536 if n >= 65536 else 1))
    bounds = [n * i // p for i in range(p + 1)]

    def work(i):
        b0, b1 = bounds[i], bounds[i + 1]
        return oracle.stats_abs(axes, [c[b0:b1] for c in coords],
                                None if weights is None else weights[b0:b1])

    with ThreadPoolExecutor(p) as ex:
        parts = list(ex.map(work, range(p)))
    out = parts[0].copy()
    for q in parts[1:]:
        out += q
    return out


def compare(got, ref, scale, unit):
    """Parity of one GPU histogram (sumw, sumw2, entries, stats) with the
    oracle's: unit-weight counts bit-exact, weighted bin sums within 1e-12
    relative, statistics within 1e-12 of max(|value|, sum of |terms|)."""
    import numpy as np
    sumw, sumw2, entries, st = got
    res = {"entries_equal": bool(entries == ref["entries"])}
    ok = res["entries_equal"]
    if unit:
        ce = bool(np.array_equal(sumw, ref["sumw"]) and np.array_equal(sumw2, ref["sumw2"]))
        res["counts_equal"] = ce
        ok = ok and ce
    else:
        for name, g, o in (("sumw", sumw, ref["sumw"]), ("sumw2", sumw2, ref["sumw2"])):
            err = np.abs(g - o)
            bad = int(np.count_nonzero(err > REL * np.abs(o)))
            nz = o != 0
            res[name + "_max_rel_err"] = float(np.max(err[nz] / np.abs(o[nz]))) if nz.any() else 0.0
            res[name + "_bins_out_of_tolerance"] = bad
            ok = ok and bad == 0
    sc = np.maximum(np.abs(ref["stats"]), scale)
    serr = np.abs(np.asarray(st) - ref["stats"]) / np.where(sc > 0, sc, 1.0)
    res["stats_max_scaled_err"] = float(np.max(serr))
    ok = ok and bool(np.all(serr <= REL))
    res["ok"] = bool(ok)
    return res


def precision_errors(sumw, sumw2, st, ref, scale):
    """Error of an approximate histogram against the binary64 oracle: per-bin
    relative error of the sums over bins the oracle fills, per statistic the
    plain relative error and the error scaled by the sum of |terms|."""
    import numpy as np
    out = {}
    for name, g, o in (("sumw", sumw, ref["sumw"]), ("sumw2", sumw2, ref["sumw2"])):
        nz = o != 0
        rel = np.abs(g[nz] - o[nz]) / np.abs(o[nz])
        out[name + "_bin_rel_err_max"] = float(rel.max()) if rel.size else 0.0
        out[name + "_bin_rel_err_median"] = float(np.median(rel)) if rel.size else 0.0
        out[name + "_empty_bins_nonzero"] = int(np.count_nonzero(g[~nz]))
    o = ref["stats"]
    g = np.asarray(st)
    out["stats_rel_err"] = [float(abs(a - b) / abs(b)) if b != 0 else float(abs(a))
                            for a, b in zip(g, o)]
    out["stats_scaled_err"] = [float(abs(a - b) / max(abs(b), s)) if max(abs(b), s) > 0 else 0.0
                               for a, b, s in zip(g, o, scale)]
    return out


# ---------------------------------------------------------------- workloads --

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


def hist_bytes(axes):
    """16 T (final sums of weights and squared weights, binary64) plus the
    edge arrays, each read once."""
    T = 1
    edges = 0
    for a in axes:
        T *= a["nbins"] + 2
        if a.get("edges") is not None:
            edges += (a["nbins"] + 1) * 8
    return 16 * T + edges


def alg_bytes(wl, n):
    """Algorithmic HBM bytes of one fill: every coordinate and weight read
    once, the final sums of weights and squared weights written once (FP64),
    each edge array read once."""
    esz = wl["coords"][0].dtype.itemsize
    per_event = len(wl["coords"]) * esz + (0 if wl["weights"] is None else esz)
    return per_event * n + hist_bytes(wl["axes"]), per_event


def to_dev(wl):
    import torch
    cols = [torch.from_numpy(c).to("cuda") for c in wl["coords"]]
    w = None if wl["weights"] is None else torch.from_numpy(wl["weights"]).to("cuda")
    return cols, w


# Events of the autotuner's sample: enough for the full-size plan's workgroups
# to run several iterations of their loop.  On 2^22 events the learned fill's
# 255 workgroups ran two, where fixed per-workgroup costs dominate, and the
# tuner at times ranked 512-thread workgroups first although they are 12%
# slower on the 5e7-event fill.
TUNE_SAMPLE = 1 << 24


def train_all(h, axes):
    for a, ax in enumerate(axes):
        if ax.get("edges") is not None:
            h.train_index(a)


def time_fills(h, step, steps, warmup):
    """Runs `step` warmup + steps times; returns the wall time of the timed
    steps and the library's kernel timing (fill and merge kernels, HIP events
    on the launch stream) summed over them."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    hs = h if isinstance(h, (list, tuple)) else [h]
    for x in hs:
        x.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fill = merge = 0.0
    launches = 0
    for x in hs:
        kt = x.timing_read()
        x.timing(False)
        fill += kt["fill_ms"]
        merge += kt["merge_ms"]
        launches += kt["launches"]
    return wall, {"fill_ms": fill / steps, "merge_ms": merge / steps, "launches": launches / steps}


def gpu_result(h):
    sumw, sumw2, entries = h.read()
    return sumw, sumw2, entries, h.stats()


def roofline(bytes_, ms):
    gbs = bytes_ / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS}


def release():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# ----------------------------------------------------------------- configs ---

def config_single(name, wl, args, threads, flags=0, compare_global=False):
    """A one-histogram workload: tuned plan timed (and the global-atomic plan
    beside it), parity of the tuned plan against the oracle."""
    import paper_2401_13310_amd as hg
    cols, w = to_dev(wl)
    n = wl["coords"][0].size
    h = hg.Hist(wl["axes"], flags)
    train_all(h, wl["axes"])
    sample = min(n, TUNE_SAMPLE)
    if args.strategy == "tuned":
        h.tune([c[:sample] for c in cols], None if w is None else w[:sample])
    else:
        h.set_strategy({"lds": hg.HIST_STRAT_LDS, "global": hg.HIST_STRAT_GLOBAL,
                        "tiled": hg.HIST_STRAT_TILED, "part": hg.HIST_STRAT_PART}[args.strategy])
    plan = h.plan_info(n, hg.HIST_F64, w is not None)
    wall, kt = time_fills(h, lambda: h.fill(cols, w), args.steps, args.warmup)
    B, per_event = alg_bytes(wl, n)
    kms = kt["fill_ms"] + kt["merge_ms"]
    out = {"workload": describe(wl, n), "plan": plan, "value": n * args.steps / wall,
           "unit": "events/s", "ms_per_step": wall / args.steps * 1e3, "kernel_ms": kms,
           "roofline": dict(roofline(B, kms), alg_bytes_per_launch=B)}
    if compare_global:
        hgb = hg.Hist(wl["axes"], flags)
        hgb.set_strategy(hg.HIST_STRAT_GLOBAL)
        sb = max(3, args.steps // 4)
        wall_g, kt_g = time_fills(hgb, lambda: hgb.fill(cols, w), sb, 1)
        kg = kt_g["fill_ms"] + kt_g["merge_ms"]
        out["global_atomics"] = {"value": n * sb / wall_g, "ms_per_step": wall_g / sb * 1e3,
                                 "kernel_ms": kg, "frac": roofline(B, kg)["frac"]}
        out["tuned_speedup_vs_global"] = out["value"] / out["global_atomics"]["value"]
        hgb.close()
    if not args.no_cpu:
        h.reset()
        h.fill(cols, w)
        got = gpu_result(h)
        ref = oracle_fill(wl["axes"], wl["coords"], wl["weights"], threads)
        scale = oracle_scale(wl["axes"], wl["coords"], wl["weights"], threads)
        out["parity"] = compare(got, ref, scale, wl["weights"] is None)
        out["cpu_oracle"] = {"value": n / ref["seconds"], "unit": "events/s",
                             "cores": ref["threads"]}
    h.close()
    del cols, w
    release()
    return out


def config_batched(args, threads):
    """64 uneven histograms: one graph replay of the persistent batch kernel,
    against 64 separate plain fills (binary search, global atomics) and 64
    separate default fills."""
    import torch

    import paper_2401_13310_amd as hg
    import synth

    members = synth.batched_64()
    cols, ws, nev, B = [], [], 0, 0
    for m in members:
        cols.append([torch.from_numpy(c).to("cuda") for c in m["coords"]])
        ws.append(torch.from_numpy(m["weights"]).to("cuda"))
        n = m["weights"].size
        nev += n
        B += n * 8 * (len(m["axes"]) + 1) + hist_bytes(m["axes"])

    def make(learned):
        hs = []
        for m in members:
            h = hg.Hist(m["axes"])
            if learned:
                train_all(h, m["axes"])
            hs.append(h)
        return hs

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    hs = make(True)
    batch = hg.Batch(hs, cols, ws)
    ms_graph = timed(lambda: batch.launch(graph=True), args.steps, args.warmup)
    plain = make(False)
    for h in plain:
        h.set_strategy(hg.HIST_STRAT_GLOBAL)
    sp = max(2, args.steps // 4)
    ms_plain = timed(lambda: [h.fill(c, w) for h, c, w in zip(plain, cols, ws)], sp, 1)
    deflt = make(True)
    ms_default = timed(lambda: [h.fill(c, w) for h, c, w in zip(deflt, cols, ws)], sp, 1)
    out = {"workload": "batched_64: 64 histograms, dims 1-3, log-uniform bins and events, "
                       "%d events, FP64 coordinates and weights" % nev,
           "value": nev / (ms_graph * 1e-3), "unit": "events/s", "ms_per_step": ms_graph,
           "kernel_ms": ms_graph,
           "roofline": dict(roofline(B, ms_graph), alg_bytes_per_launch=B,
                            kernel="batch graph (persistent kernel + partition passes)"),
           "plain_fills": {"value": nev / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                           "what": "64 hist_fill calls, binary search, global atomics"},
           "default_fills": {"value": nev / (ms_default * 1e-3), "ms_per_step": ms_default,
                             "what": "64 hist_fill calls, learned index, heuristic plans"},
           "speedup_vs_plain": ms_plain / ms_graph}
    for h in plain + deflt:
        h.close()
    if not args.no_cpu:
        for h in hs:
            h.reset()
        batch.launch(graph=True)
        torch.cuda.synchronize()
        got = [gpu_result(h) for h in hs]

        def ref_of(i):
            m = members[i]
            r = oracle_fill(m["axes"], m["coords"], m["weights"], 1)
            s = oracle_scale(m["axes"], m["coords"], m["weights"], 1)
            return r, s

        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            refs = list(ex.map(ref_of, range(len(members))))
        dt = time.perf_counter() - t0
        per = [compare(g, r, s, False) for g, (r, s) in zip(got, refs)]
        out["parity"] = {"members": len(per), "members_ok": sum(p["ok"] for p in per),
                         "ok": all(p["ok"] for p in per),
                         "sumw_max_rel_err": max(p["sumw_max_rel_err"] for p in per),
                         "stats_max_scaled_err": max(p["stats_max_scaled_err"] for p in per)}
        out["cpu_oracle"] = {"value": nev / dt, "unit": "events/s", "cores": threads,
                             "what": "one oracle per member, members in parallel (with the "
                                     "statistics-scale pass)"}
    batch.close()
    for h in hs:
        h.close()
    del cols, ws
    release()
    return out


def config_precision(args, threads):
    """2e8 FP32 events in 12 slices of 2^24 into 1e4 fixed bins: the
    compensated FP32 accumulator against the all-binary64 path on the same
    values widened, both against the binary64 oracle."""
    import numpy as np
    import torch

    import paper_2401_13310_amd as hg
    import synth

    axes = synth.precision_axes()
    slices = list(synth.precision_slices())
    n = sum(x.size for x, _ in slices)
    xs32 = [torch.from_numpy(x).to("cuda") for x, _ in slices]
    ws32 = [torch.from_numpy(w).to("cuda") for _, w in slices]
    xs64 = [x.double() for x in xs32]
    ws64 = [w.double() for w in ws32]
    out = {"workload": "precision: 10000 fixed bins [0, 100); %d events x ~ Gamma(2, 10), "
                       "w ~ LogNormal(0, 2), FP32, %d slices of up to 2^24" % (n, len(slices))}
    hs = {}
    for key, flags, xs, ws, esz in (("f32c", hg.HIST_F_ACC_F32C, xs32, ws32, 4),
                                    ("f64", 0, xs64, ws64, 8)):
        h = hg.Hist(axes, flags)
        sample = min(xs[0].numel(), 1 << 22)
        h.tune([xs[0][:sample]], ws[0][:sample])

        def step(h=h, xs=xs, ws=ws):
            for x, w in zip(xs, ws):
                h.fill([x], w)

        steps = max(3, args.steps // 4)
        wall, kt = time_fills(h, step, steps, 1)
        B = n * 2 * esz + 12 * hist_bytes(axes)
        kms = kt["fill_ms"] + kt["merge_ms"]
        out[key] = {"value": n * steps / wall, "unit": "events/s",
                    "ms_per_step": wall / steps * 1e3, "kernel_ms": kms,
                    "roofline": dict(roofline(B, kms), alg_bytes_per_launch=B),
                    "plan": h.plan_info(xs[0].numel(), hg.HIST_F32 if esz == 4 else hg.HIST_F64,
                                        True)}
        hs[key] = (h, step)
    out["f32c_speedup_vs_f64"] = out["f32c"]["value"] / out["f64"]["value"]
    if not args.no_cpu:
        # the binary64 oracle on the widened values, one oracle per slice
        def work(i):
            x, w = slices[i]
            r = oracle_fill(axes, [x], w, 1)
            s = oracle_scale(axes, [x], w, 1)
            return r, s

        t0 = time.perf_counter()
        with ThreadPoolExecutor(min(threads, len(slices))) as ex:
            parts = list(ex.map(work, range(len(slices))))
        dt = time.perf_counter() - t0
        ref = {"sumw": sum(p[0]["sumw"] for p in parts), "sumw2": sum(p[0]["sumw2"] for p in parts),
               "stats": sum(p[0]["stats"] for p in parts),
               "entries": sum(p[0]["entries"] for p in parts)}
        scale = sum(p[1] for p in parts)
        out["cpu_oracle"] = {"value": n / dt, "unit": "events/s",
                             "cores": min(threads, len(slices))}
        for key, (h, step) in hs.items():
            h.reset()
            step()
            got = gpu_result(h)
            out[key]["errors_vs_fp64_oracle"] = precision_errors(got[0], got[1], got[3], ref,
                                                                 scale)
            if key == "f64":
                out[key]["parity"] = compare(got, ref, scale, False)
            else:
                out[key]["entries_equal"] = bool(got[2] == ref["entries"])
    for h, _ in hs.values():
        h.close()
    del xs32, ws32, xs64, ws64
    release()
    return out


# ------------------------------------------------------- counter ingestion --

def load_traffic(path, workload, n, plan):
    """HBM bytes per fill launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy
    of known size), if measured on the current kernel sources and plan."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(workload)
    if (not rec or rec.get("events") != n or rec.get("source_hash") != kernel_source_hash()
            or rec.get("plan") != plan):
        return None
    return rec.get("bytes_per_launch")


def _counter_per_dispatch(path, counter, last=None):
    """{kernel name: [value per dispatch]} for one counter, from rocprofv3's
    counter_collection.csv or its rocpd database; `last`, if given, receives
    each kernel's last dispatch id."""
    per = {}
    rows = []
    if path.endswith(".csv"):
        import csv
        sums = {}
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                key = (int(row["Dispatch_Id"]), row["Kernel_Name"])
                sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
        rows = [(disp, kname, val) for (disp, kname), val in sorted(sums.items())]
    else:
        import sqlite3
        db = sqlite3.connect(path)
        rows = list(db.execute(
            "select dispatch_id, kernel_name, sum(value) from counters_collection "
            "where counter_name = ? group by dispatch_id, kernel_name order by dispatch_id",
            (counter,)))
    for disp, kname, val in rows:
        per.setdefault(kname, []).append(val)
        if last is not None:
            last[kname] = max(last.get(kname, -1), int(disp))
    return per


def ingest(args):
    lastd = {}
    fetch = _counter_per_dispatch(args.ingest[0], "FETCH_SIZE", lastd)
    write = _counter_per_dispatch(args.ingest[1], "WRITE_SIZE")
    # calibration: the elementwise copy the profile run makes last (reads and
    # writes one column); the runtime's own copy kernels also move host data
    copy = [k for k in fetch if "elementwise" in k.lower() and "hg::" not in k and k in write]
    # the fill kernel: the one the profile run's timed fills (after tuning)
    # launched last
    fill = [k for k in fetch if k in write and
            ("fill_kernel" in k or "fill_learned_kernel" in k or "fill_shape_kernel" in k)]
    if not copy or not fill:
        raise SystemExit("ingest: need the fill kernel and the calibration copy in both runs")
    wl = build_workload(args.workload, args.events)
    n = wl["coords"][0].size
    known = n * wl["coords"][0].dtype.itemsize            # bytes read and written by each copy
    ck = copy[-1]
    f_copy = sorted(fetch[ck][-3:])[len(fetch[ck][-3:]) // 2] * 1024.0
    w_copy = sorted(write[ck][-3:])[len(write[ck][-3:]) // 2] * 1024.0
    fk = max(fill, key=lambda k: lastd[k])
    last = max(1, args.steps)                 # the fills after tuning are the last ones
    fv, wv = sorted(fetch[fk][-last:]), sorted(write[fk][-last:])
    f_fill = fv[len(fv) // 2] * 1024.0
    w_fill = wv[len(wv) // 2] * 1024.0
    # its merge kernel (staged merge), launched right after it
    merge = [k for k in fetch if k in write and "stage_reduce" in k and lastd[k] > lastd[fk]]
    mk = min(merge, key=lambda k: lastd[k]) if merge else None
    f_merge = w_merge = 0.0
    if mk:
        mv, mw = sorted(fetch[mk][-last:]), sorted(write[mk][-last:])
        f_merge, w_merge = mv[len(mv) // 2] * 1024.0, mw[len(mw) // 2] * 1024.0
    sf, sw = known / f_copy, known / w_copy
    with open(args.ingest[2]) as f:
        prof = json.load(f)
    if prof.get("source_hash") != kernel_source_hash() or prof.get("events") != n:
        raise SystemExit("ingest: the profile run used other kernel sources or sizes")
    rec = {"events": n, "kernel": fk, "source_hash": kernel_source_hash(), "plan": prof["plan"],
           "fetch_kib_raw": f_fill / 1024.0, "write_kib_raw": w_fill / 1024.0,
           "merge_kernel": mk, "merge_fetch_kib_raw": f_merge / 1024.0,
           "merge_write_kib_raw": w_merge / 1024.0,
           "copy_kernel": ck, "copy_bytes": known, "fetch_scale": sf, "write_scale": sw,
           "fill_bytes_per_launch": f_fill * sf + w_fill * sw,
           "bytes_per_launch": (f_fill + f_merge) * sf + (w_fill + w_merge) * sw}
    try:
        with open(args.traffic) as f:
            allrec = json.load(f)
    except (OSError, ValueError):
        allrec = {}
    allrec[args.workload] = rec
    with open(args.traffic, "w") as f:
        json.dump(allrec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


# -------------------------------------------------------------------- main ---

def run_single(args, wl, headline):
    """Times one workload (the headline runs its configs and CPU legs too)."""
    import numpy as np
    import torch

    import paper_2401_13310_amd as hg

    n = wl["coords"][0].size
    threads = cpu_threads()
    log("workload %s, %d events" % (wl["name"], n))
    cols, w = to_dev(wl)
    f32 = wl["coords"][0].dtype == np.float32
    flags = hg.HIST_F_ACC_F32C if wl["name"] == "precision" else 0
    variable = any(a.get("edges") is not None for a in wl["axes"])

    h = hg.Hist(wl["axes"], flags)
    train_ms = None
    if variable:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        train_all(h, wl["axes"])
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
    sample = min(n, TUNE_SAMPLE)
    if args.strategy == "tuned":
        h.tune([c[:sample] for c in cols], None if w is None else w[:sample])
    else:
        h.set_strategy({"lds": hg.HIST_STRAT_LDS, "global": hg.HIST_STRAT_GLOBAL,
                        "tiled": hg.HIST_STRAT_TILED, "part": hg.HIST_STRAT_PART}[args.strategy])
    plan = h.plan_info(n, hg.HIST_F32 if f32 else hg.HIST_F64, w is not None)
    if args.profile:
        for _ in range(args.steps):
            h.fill(cols, w)
        torch.cuda.synchronize()
        dst = torch.empty_like(cols[0])
        for _ in range(3):
            dst.copy_(cols[0])                 # reads and writes n * itemsize bytes
        for _ in range(3):
            torch.mul(cols[0], 1.0, out=dst)   # the same traffic, as a plain kernel
        torch.cuda.synchronize()
        print("profile run: %d fills of %d events, plan %s; copy of %d bytes x3; sources %s"
              % (args.steps, n, plan, cols[0].numel() * cols[0].element_size(),
                 kernel_source_hash()), flush=True)
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        tag = args.workload if args.strategy == "tuned" else "%s_%s" % (args.workload, args.strategy)
        with open(os.path.join(ROOT, "gpurun_out", "profile_plan_%s.json" % tag), "w") as f:
            json.dump({"workload": args.workload, "events": n, "plan": plan,
                       "source_hash": kernel_source_hash()}, f)
        h.close()
        return

    wall, kt = time_fills(h, lambda: h.fill(cols, w), args.steps, args.warmup)
    log("timed %d steps: %.4f ms/step" % (args.steps, wall / args.steps * 1e3))
    ms_step = wall / args.steps * 1e3
    value = n * args.steps / wall
    fill_ms = kt["fill_ms"] / max(1.0, kt["launches"]) if kt["launches"] else ms_step
    merge_ms = kt["merge_ms"] / max(1.0, kt["launches"]) if kt["launches"] else 0.0
    kernel_ms = fill_ms + merge_ms
    B, per_event = alg_bytes(wl, n)
    traffic = load_traffic(args.traffic, args.workload, n, plan)
    rl = roofline(B, kernel_ms)
    rl.update({"traffic": traffic, "kernel": "the fill kernel + its staged merge kernel (one hist_fill)",
               "kernel_ms": kernel_ms, "fill_kernel_ms": fill_ms, "merge_kernel_ms": merge_ms,
               "alg_bytes_per_launch": B, "alg_bytes_per_event": per_event})
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
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic (seeded numpy PCG64), resident in HBM before timing",
        "config": {"workload": describe(wl, n),
                   "search": "learned" if variable else "fixed-width formula",
                   "plan": plan},
        "roofline": rl,
        "step_hbm_frac": B / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    if train_ms is not None:
        out["index_train_ms"] = train_ms
    if headline:
        out["probes"] = probes(cols[0])
        read_gbs = out["probes"]["read_GBps"]
        rl["achievable_read_GBps"] = read_gbs
        rl["frac_of_achievable_read"] = rl["achieved"] / read_gbs if read_gbs > 0 else None
    if variable and not args.no_bsearch:
        hb = hg.Hist(wl["axes"], flags)
        hb.tune([c[:sample] for c in cols], None if w is None else w[:sample])
        steps_b = max(3, args.steps // 2)
        wall_b, kt_b = time_fills(hb, lambda: hb.fill(cols, w), steps_b, 1)
        out["bsearch"] = {"value": n * steps_b / wall_b, "ms_per_step": wall_b / steps_b * 1e3,
                          "kernel_ms": kt_b["fill_ms"] / max(1.0, kt_b["launches"]) +
                          kt_b["merge_ms"] / max(1.0, kt_b["launches"]),
                          "plan": hb.plan_info(n, hg.HIST_F64, w is not None)}
        out["learned_speedup_vs_bsearch"] = out["value"] / out["bsearch"]["value"]
        hb.close()
    if not args.no_cpu:
        # the timed plan's result: one more fill after a reset
        h.reset()
        h.fill(cols, w)
        got = gpu_result(h)
        log("CPU oracle, one thread, %d events" % n)
        ref = oracle_fill(wl["axes"], wl["coords"], wl["weights"], 1)
        log("CPU oracle, %d threads" % threads)
        ref_all = oracle_fill(wl["axes"], wl["coords"], wl["weights"], threads)
        scale = oracle_scale(wl["axes"], wl["coords"], wl["weights"], threads)
        out["parity"] = compare(got, ref, scale, w is None)
        out["parity"]["what"] = ("the timed plan (reset, one fill) against the sequential oracle "
                                 "on the same %d events" % n)
        out["cpu_baseline"] = {
            "value": n / ref["seconds"], "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": "one full step (%d events, the same arrays), sequential C oracle, %.2f s"
                      % (n, ref["seconds"]),
            "cpu_model": cpu_model(),
            "all_cores": {"value": n / ref_all["seconds"], "unit": "events/s",
                          "cores": ref_all["threads"],
                          "what": "the same oracle on %d contiguous chunks in parallel threads, "
                                  "summed in chunk order, %.2f s"
                                  % (ref_all["threads"], ref_all["seconds"]),
                          "counts_equal_sequential": bool(
                              np.array_equal(ref_all["sumw"], ref["sumw"]))},
        }
    h.close()
    del cols, w
    release()
    if headline:
        threads = cpu_threads()
        wanted = [c.strip() for c in args.configs.split(",") if c.strip()]
        configs = {}
        for c in wanted:
            log("config %s" % c)
            try:
                if c == "C1":
                    configs["C1_plain_1d"] = config_single("C1", build_workload("plain_1d", 0),
                                                           args, threads)
                elif c == "C3":
                    configs["C3_corr_3d"] = config_single("C3", build_workload("corr_3d", 0), args,
                                                          threads, compare_global=True)
                elif c == "C4":
                    configs["C4_batched_64"] = config_batched(args, threads)
                elif c == "C5":
                    configs["C5_precision"] = config_precision(args, threads)
                elif c == "F1":
                    configs["F1_host_ingest"] = config_host(args)
                elif c == "F2":
                    configs["F2_multi_pass"] = config_multi(args, threads)
                else:
                    raise SystemExit("unknown config %s" % c)
            except (RuntimeError, ValueError, MemoryError) as e:
                configs[c] = {"error": "%s: %s" % (type(e).__name__, e)}
            log("config %s done" % c)
        if configs:
            out["configs"] = configs
    print(json.dumps(out), flush=True)


def probes(col):
    """The ceilings of the roofline, measured with the library's probes on
    this GPU: streaming read bandwidth (over the workload's own column), LDS
    atomic rates (u32 and binary64 adds, one 1024-thread workgroup per CU)
    and device-scope atomic rates without return (u64 and binary64 adds to
    hashed addresses of a 64 MiB array)."""
    import torch

    import paper_2401_13310_amd as hg
    stream = torch.cuda.current_stream().cuda_stream
    nbytes = col.numel() * col.element_size()
    out = {"read_GBps": hg.hist_probe(hg._lib.HIST_PROBE_READ, col.data_ptr(), nbytes, 10,
                                      stream)["rate"] / 1e9,
           "read_bytes": nbytes}
    clk = 2.4e9
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for name, kind in (("lds_u32", hg._lib.HIST_PROBE_LDS_U32), ("lds_f64", hg._lib.HIST_PROBE_LDS_F64)):
        r = hg.hist_probe(kind, None, 0, 5, stream)["rate"]
        out[name + "_Gops"] = r / 1e9
        out[name + "_lanes_per_clk_per_cu"] = r / clk / cus
    buf = torch.zeros(8 << 20, dtype=torch.float64, device="cuda")
    for name, kind in (("global_u64", hg._lib.HIST_PROBE_GLOBAL_U64),
                       ("global_f64", hg._lib.HIST_PROBE_GLOBAL_F64)):
        out[name + "_Gops"] = hg.hist_probe(kind, buf.data_ptr(), buf.numel() * 8, 5,
                                            stream)["rate"] / 1e9
    del buf
    out["what"] = ("hist_probe kernels timed with HIP events; per-CU rates assume the 2.4 GHz "
                   "peak clock and %d CUs" % cus)
    return out


def _event_ms(fn, reps):
    """Mean milliseconds of fn() between HIP events on the current stream
    (host-synchronous calls included)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def config_host(args):
    """Events in host memory (hist_fill_host) on the variable-bin workload:
    pageable and page-locked input against the measured host-to-device copy
    rate of the same bytes; counts against a device-resident fill."""
    import numpy as np
    import torch

    import paper_2401_13310_amd as hg
    wl = build_workload("variable_1d", 0)
    x = wl["coords"][0]
    n = x.size
    nbytes = x.nbytes
    reps = max(2, min(args.steps, 5))
    xp = torch.from_numpy(x).pin_memory()
    xh = torch.from_numpy(x)
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    pinned_copy_ms = _event_ms(lambda: dst.copy_(xp, non_blocking=True), reps)
    pageable_copy_ms = _event_ms(lambda: dst.copy_(xh), reps)
    ref = hg.Hist(wl["axes"])
    train_all(ref, wl["axes"])
    ref.fill([dst])
    rs, _, re_, rst = gpu_result(ref)
    out = {"workload": describe(wl, n), "bytes": nbytes,
           "h2d_pinned_GBps": nbytes / (pinned_copy_ms * 1e-3) / 1e9,
           "h2d_pageable_GBps": nbytes / (pageable_copy_ms * 1e-3) / 1e9}
    for name, cols, pinned in (("pageable", [x], False), ("pinned", [xp], True)):
        h = hg.Hist(wl["axes"])
        train_all(h, wl["axes"])
        h.fill_host(cols, pinned=pinned)          # slots and scratch
        h.reset()
        ms = _event_ms(lambda: h.fill_host(cols, pinned=pinned), reps)
        h.reset()
        h.fill_host(cols, pinned=pinned)
        s, _, e, st = gpu_result(h)
        out[name] = {"ms_per_fill": ms, "events_per_s": n / (ms * 1e-3),
                     "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "frac_of_pinned_h2d": (nbytes / (ms * 1e-3) / 1e9) /
                                           out["h2d_pinned_GBps"],
                     "counts_equal_device_fill": bool(np.array_equal(s, rs)) and e == re_,
                     "stats_max_rel_diff": float(np.max(np.abs(st - rst) /
                                                        np.maximum(np.abs(rst), 1e-300)))}
        h.close()
    ref.close()
    del xp, xh, dst
    release()
    return out


def config_multi(args, threads):
    """One pass over the correlated 3D columns filling four histograms (the
    three 1D projections and r = sqrt(x^2+y^2+z^2) of the events with z > 0)
    against the same projections filled one by one; every member against the
    oracle of its defined events."""
    import numpy as np
    import torch

    import oracle
    from oracle import expr as E
    import paper_2401_13310_amd as hg
    wl = build_workload("corr_3d", 0)
    n = len(wl["coords"][0])
    names = ["x", "y", "z"]
    cols, _ = to_dev(wl)
    ax1 = [{"nbins": 100, "xmin": -4.0, "xmax": 4.0}]
    members = [(ax1, {"coords": ["x"]}), (ax1, {"coords": ["y"]}), (ax1, {"coords": ["z"]}),
               ([{"nbins": 200, "xmin": 0.0, "xmax": 8.0}],
                {"filter": "z > 0", "coords": ["sqrt(x*x + y*y + z*z)"]})]
    hists = [hg.Hist(a) for a, _ in members]
    plan = hg.Multi(hists, [d for _, d in members], names)
    reps = max(2, min(args.steps, 10))
    multi_ms = _event_ms(lambda: plan.fill(cols), reps)
    # the same four histograms without the shared pass: three plain fills,
    # and r computed and filtered by torch, then filled
    plain = [hg.Hist(ax1) for _ in range(3)]
    hr = hg.Hist(members[3][0])

    def separate():
        for hh, c in zip(plain, cols):
            hh.fill([c])
        x, y, z = cols
        r = torch.sqrt(x * x + y * y + z * z)[z > 0]
        hr.fill([r])
    sep_ms = _event_ms(separate, reps)
    proj_plan = hg.Multi([hg.Hist(ax1) for _ in range(3)], [{"coords": [nm]} for nm in names], names)
    proj_ms = _event_ms(lambda: proj_plan.fill(cols), reps)
    plain_ms = _event_ms(lambda: [hh.fill([c]) for hh, c in zip(plain, cols)], reps)
    for hh in hists:
        hh.reset()
    plan.fill(cols)
    torch.cuda.synchronize()
    ok = True
    worst = 0.0
    for hh, (axes, d) in zip(hists, members):
        ops = {"filter": hg.parse(d["filter"], names) if d.get("filter") else None,
               "coords": [hg.parse(c, names) for c in d["coords"]]}
        oc, ow = E.apply_define(ops, wl["coords"], len(axes))
        s, _, e, st = gpu_result(hh)
        ref = oracle_fill(axes, oc, ow, threads)
        scale = oracle_scale(axes, oc, ow, threads)
        ok = ok and e == ref["entries"] and bool(np.array_equal(s, ref["sumw"]))
        worst = max(worst, float(np.max(np.abs(st - ref["stats"]) /
                                        np.maximum(np.maximum(np.abs(ref["stats"]), scale), 1e-300))))
        ok = ok and worst <= REL
    bytes_ = 3 * 8 * n + sum(hist_bytes(a) for a, _ in members)
    out = {"workload": "corr_3d columns, %d events: 1D projections x, y, z and r = sqrt(x^2+y^2+z^2)"
                       " for z > 0 in one pass" % n,
           "multi_pass_ms": multi_ms, "events_per_s": n / (multi_ms * 1e-3),
           "roofline": roofline(bytes_, multi_ms),
           "separate_ms": sep_ms,
           "separate_what": "three plain hist_fill calls, then r = sqrt(x*x+y*y+z*z)[z > 0] in "
                            "torch and a fourth hist_fill",
           "speedup_vs_separate": sep_ms / multi_ms,
           "projections_multi_pass_ms": proj_ms,
           "projections_plain_fills_ms": plain_ms,
           "projections_speedup": plain_ms / proj_ms,
           "parity": {"ok": ok, "stats_max_scaled_err": worst,
                      "what": "every member: counts bit-exact, entries equal, statistics 1e-12"}}
    for o in (plan, proj_plan):
        o.close()
    del cols
    release()
    return out


def sweep(args):
    """The paper's launch-shape questions (Sec. 4.3) on gfx950: events per
    thread of the fill kernel (1, 2, 4, 8) with fused statistics, and the
    statistics as separate reduction kernels (one per statistic, re-reading
    the columns; 1, 4, 16 events per thread) against fused.  One-axis
    binary64 workloads: plain_1d at 2^27 events (fixed-width, weighted), the
    variable-bin workload (learned index, 5e7) and the paper's own shape (1000
    edges on [0, 1], x ~ U[0, 1], 5e7, edges in LDS).  Every variant's counts
    are compared bit for bit with the default shape's, and its statistics
    within 1e-12 of the default's scale."""
    import numpy as np
    import paper_2401_13310_amd as hg
    import synth
    cases = [("plain_1d_2e27", synth.plain_1d(1 << 27)),
             ("variable_1d", synth.variable_1d(synth.VARIABLE_1D_N)),
             ("paper_1d", synth.paper_1d(50_000_000))]
    out = []
    for name, wl in cases:
        n = len(wl["coords"][0])
        cols, w = to_dev(wl)
        bytes_, _ = alg_bytes(wl, n)
        ref = None
        rows = []
        shapes = [(0, 0)] + [(u, 0) for u in (1, 2, 4, 8)] + [(0, e) for e in (1, 4, 16)]
        for unroll, ept in shapes:
            h = hg.Hist(wl["axes"])
            train_all(h, wl["axes"])
            h.set_shape(unroll, ept)
            shape = h.plan_shape(n, weighted=w is not None)
            step = lambda: h.fill(cols, w)
            wall, kt = time_fills(h, step, args.steps, args.warmup)
            ms = kt["fill_ms"] + kt["merge_ms"]
            h.reset()
            h.fill(cols, w)
            sumw, _, entries, st = gpu_result(h)
            row = {"unroll": shape["unroll"], "stats": "fused" if shape["stats_ept"] == 0 else
                   "separate, %d events/thread" % shape["stats_ept"],
                   "requested": [unroll, ept], "kernel_ms": ms,
                   "ms_per_step": wall * 1e3 / args.steps, "events_per_s": n / (ms * 1e-3),
                   "frac": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if ref is None:
                ref = (sumw, entries, st)
                row["default"] = True
            else:
                scale = np.maximum(np.abs(ref[2]), 1e-300)
                row["counts_equal_default"] = bool(np.array_equal(sumw, ref[0]) if w is None
                                                   else np.allclose(sumw, ref[0], rtol=1e-12, atol=0))
                row["entries_equal_default"] = entries == ref[1]
                row["stats_max_rel_diff"] = float(np.max(np.abs(st - ref[2]) / scale))
            log("sweep %s unroll=%d stats_ept=%d: %.4f ms" % (name, shape["unroll"],
                                                               shape["stats_ept"], ms))
            rows.append(row)
            h.close()
        fused = [r for r in rows if r["stats"] == "fused"]
        sep = [r for r in rows if r["stats"] != "fused"]
        best_f = min(fused, key=lambda r: r["kernel_ms"])
        worst_f = max(fused, key=lambda r: r["kernel_ms"])
        best_s = min(sep, key=lambda r: r["kernel_ms"])
        out.append({"workload": describe(wl, n), "alg_bytes": bytes_, "rows": rows,
                    "best_unroll": best_f["unroll"],
                    "best_vs_worst_unroll": worst_f["kernel_ms"] / best_f["kernel_ms"],
                    "fused_vs_separate": best_s["kernel_ms"] / best_f["kernel_ms"]})
        del cols, w
        release()
    print(json.dumps({"sweep": out, "steps": args.steps, "warmup": args.warmup}), flush=True)


def main():
    args = parse()
    if args.ingest:
        ingest(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "sweep":
        sweep(args)
        return
    if args.workload == "batched_64":
        out = config_batched(args, cpu_threads())
        out.update({"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": "f64", "data": "synthetic (seeded numpy PCG64)",
                    "config": {"workload": out.pop("workload")}})
        print(json.dumps(out), flush=True)
        return
    run_single(args, build_workload(args.workload, args.events),
               headline=args.workload == "variable_1d" and not args.events)


if __name__ == "__main__":
    main()
