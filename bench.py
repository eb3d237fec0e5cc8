#!/usr/bin/env python3
"""Throughput of the per-level AMR hydro step on one MI355X.

Workload: the 256^3 periodic box (level 8, 2,097,152 octs, 16,777,216 cells)
with seeded lognormal density and Mach-2 k^-2 random velocities, gamma 5/3,
CFL 0.8 (the roofline configuration).  One timed step is the whole hot path:
key encode + radix sort + level ranges, FNV hash rebuild, neighbour lists,
CFL dt, the hydro update of every level, coarse-fine correction and
restriction (the last two are empty on a single level).  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line.  `value` is FP64 cell-updates/s; the mixed form
(FP32 reconstruction/HLLC, FP64 state) is reported under "mixed".
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hydro cell-updates/s on 1 MI355X, FP64 vs mixed FP32; % of HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell-update of the hydro kernel: read uold (40 B),
# write unew (40 B), the 27-entry int32 neighbour list over 8 cells (13.5 B)
ALG_BYTES_PER_CELL = 93.5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hydro_traffic_random256.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("rg_brick.hip", "rg_brick.hpp", "rg_math.hpp", "rg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2607_20704_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(form):
    """HBM bytes per hydro launch from the committed counter summary, or None
    when it is missing or the kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_digest():
        return None
    m = re.search(r"traffic_bytes_per_launch_%s:\s*([0-9.eE+]+)" % form, text)
    return float(m.group(1)) if m else None


def time_form(D, u0, w, form, steps, warmup, api):
    import torch
    a, b = u0.clone(), torch.empty_like(u0)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    flags = api.L.RG_STEP_REKEY | api.RG_STEP_REBUILD

    def one_step(a, b, h0=None, h1=None):
        D.prepare(flags)
        api.cfl_dt(a, D.son_mask, D.level_begin, D.lmin, D.lmax, w.gamma, w.cfl, dt)
        if h0 is not None:
            h0.record()
        for l in range(D.lmin, D.lmax + 1):
            D.hydro_level(l, dt, w.gamma, a, b, form)
        if h1 is not None:
            h1.record()
        if D.lmax > D.lmin:
            api.apply_coarse_corrections(b, D.corr, D.corr_base, D.nbr27, D.corr_base, D.n)
            for l in range(D.lmax, D.lmin, -1):
                api.restrict_level(b, D.father_cell, int(D.level_begin[l]), int(D.level_begin[l + 1]))

    for _ in range(warmup):
        one_step(a, b)
        a, b = b, a
    torch.cuda.synchronize()
    h0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    h1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for k in range(steps):
        one_step(a, b, h0[k], h1[k])
        a, b = b, a
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / steps
    hydro_ms = sum(x.elapsed_time(y) for x, y in zip(h0, h1)) / steps
    # hydro-only steps (dt + update with prebuilt lists), for the paper's
    # "Godunov solver only" comparison
    s2, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s2.record()
    for k in range(steps):
        api.cfl_dt(a, D.son_mask, D.level_begin, D.lmin, D.lmax, w.gamma, w.cfl, dt)
        for l in range(D.lmin, D.lmax + 1):
            D.hydro_level(l, dt, w.gamma, a, b, form)
        a, b = b, a
    e2.record()
    torch.cuda.synchronize()
    hydro_only_ms = s2.elapsed_time(e2) / steps
    return {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "hydro_kernel_ms": hydro_ms,
            "hydro_only_ms_per_step": hydro_only_ms, "state": a}


def cpu_baseline(w, sample_octs):
    """The oracle, as it stands, on the host: its hydro update (tile,
    reconstruction, Riemann, update) of the first `sample_octs` octs in key
    order, with its own neighbour lists."""
    import numpy as np

    from oracle import oracle as O
    T = O.Tree(w.ijkl, w.bc)
    u = T.permute_cells(w.u)
    dt = T.cfl_dt(u, w.gamma, w.cfl)
    unew = np.zeros_like(u)
    corr = np.zeros(1)
    n = min(sample_octs, T.n)
    t0 = time.perf_counter()
    O.hydro_octs(T.ijkl, T.nbr27, T.son_mask, 0, n, u, unew, corr, dt, w.gamma)
    sec = time.perf_counter() - t0
    return {"value": 8 * n / sec, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "hydro update (stencil, MUSCL-Hancock, HLLC, update) of the first %d octs (%d cells, a "
                      "Hilbert-contiguous %s of the box) of the same 256^3 state; serial FP64, %.1f s"
                      % (n, 8 * n, "half" if 2 * n == T.n else "part", sec)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-octs", type=int, default=1 << 20)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d requested)" % args.gpus)

    import numpy as np
    import torch

    from paper_2607_20704_amd import api, inputs
    torch.cuda.set_device(0)
    log("generating the 256^3 random-field box")
    w = inputs.random_uniform()
    D = api.DeviceTree(w.ijkl, w.bc)
    u0 = D.to_key_order(w.u)
    torch.cuda.synchronize()
    cells = 8 * D.n
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    res = {}
    for f in forms:
        form = api.RG_FP64 if f == "fp64" else api.RG_MIXED
        log("timing form %s: %d warmup + %d steps" % (f, args.warmup, args.steps))
        res[f] = time_form(D, u0, w, form, args.steps, args.warmup, api)
        log("  %.3f ms/step, hydro kernel %.3f ms" % (res[f]["ms_per_step"], res[f]["hydro_kernel_ms"]))

    def roof(r, f):
        achieved = ALG_BYTES_PER_CELL * cells / (r["hydro_kernel_ms"] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f),
                "kernel": "k_hydro_brick", "alg_bytes_per_launch": ALG_BYTES_PER_CELL * cells,
                "kernel_ms": round(r["hydro_kernel_ms"], 4)}

    def summary(r, f):
        return {"value": cells / (r["ms_per_step"] * 1e-3), "ms_per_step": round(r["ms_per_step"], 4),
                "hydro_only_cell_updates_per_s": cells / (r["hydro_only_ms_per_step"] * 1e-3),
                "hydro_only_ms_per_step": round(r["hydro_only_ms_per_step"], 4),
                "ns_per_cell": r["ms_per_step"] * 1e6 / cells, "roofline": roof(r, f)}

    primary = "fp64" if "fp64" in res else forms[0]
    out = {"metric": METRIC, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if primary == "fp64" else "f32-flux/f64-state", "data": "synthetic"}
    s = summary(res[primary], primary)
    out["value"] = s["value"]
    out["ms_per_step"] = s["ms_per_step"]
    out["config"] = {"workload": "random_uniform_l8: 256^3 periodic box, lognormal rho (sigma_ln 0.5), k^-2 "
                                 "velocities at rms Mach 2, p=1, gamma 5/3, CFL 0.8, seed 20704",
                     "octs": D.n, "cells": cells, "levels": [D.lmin, D.lmax], "form": primary,
                     "schedule": {str(l): {"bricks": c[0], "per_oct": c[1]} for l, c in D.schedule_counts().items()},
                     "step": "rekey+sort+hash+neighbours+dt+hydro(+corrections+restriction)"}
    out["roofline"] = s["roofline"]
    out["hydro_only_cell_updates_per_s"] = s["hydro_only_cell_updates_per_s"]
    out["ns_per_cell"] = s["ns_per_cell"]
    for f in forms:
        if f != primary:
            out[f] = summary(res[f], f)
            out[f]["dtype"] = "f32-flux/f64-state" if f == "mixed" else "f64"
    if "fp64" in res and "mixed" in res:
        a, b = res["fp64"]["state"], res["mixed"]["state"]
        l1 = ((a - b).abs().sum(0) / a.abs().sum(0).clamp_min(1e-300)).cpu().numpy()
        out["mixed"]["l1_vs_fp64_after_%d_steps" % (2 * args.steps + args.warmup)] = [float(x) for x in l1]
    if not args.no_cpu_baseline:
        log("oracle CPU baseline on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_octs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
