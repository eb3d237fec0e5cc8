#!/usr/bin/env python3
"""Throughput of the per-level AMR hydro step on one MI355X.

Workload: the 256^3 periodic box (level 8, 2,097,152 octs, 16,777,216 cells)
with seeded lognormal density and Mach-2 k^-2 random velocities, gamma 5/3,
CFL 0.8 (the roofline configuration).  One timed step is the whole hot path:
FNV hash rebuild from the keys, neighbour lists, CFL dt, the hydro update of
every level, coarse-fine correction and restriction (the last two are empty
on a single level).  Re-keying (key encode, radix sort, level ranges; needed
only when the tree changes) is timed separately as "rekey_ms".  Inputs are
resident in HBM before the timed region starts.  Each figure is the median
of 5 repetitions of exactly --steps steps.

Prints one JSON line.  `value` is FP64 cell-updates/s; the mixed form
(FP32 reconstruction/HLLC, FP64 state) is reported under "mixed".  Beside
it: "sedov_amr" (global steps of the Sedov blast on its graded AMR tree,
both forms), "batched" (64 seeded boxes of uneven size and depth, 20 steps
in one graph launch, against the same boxes stepped one at a time),
"deep_amr" (clumpy gas on a base-7 tree refined to level 12, about 28 M
cells), "mg_poisson" and "dynamic" (refinement on the device).  The kernel
variants are chosen by the autotuner before timing (they give identical
bits).  "cpu_baseline" times the oracle on the host (its OpenMP build on
every core and its serial build) and "parity" compares the device's state
after the same steps, in the timed launch shape, with the oracle's: FP64
within 1e-12 per cell, the mixed form within an L1 of 1e-5 per field.  A
mismatch prints the line with a null value and exits non-zero.
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
REPS = 5
# algorithmic bytes per cell-update of the hydro kernel: read uold (40 B),
# write unew (40 B), the 27-entry int32 neighbour list over 8 cells (13.5 B)
ALG_BYTES_PER_CELL = 93.5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hydro_traffic_random256.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest():
    """Digest of the brick kernel's code (its sources without comments and
    blank lines, so that a comment edit keeps the counter summary valid)."""
    h = hashlib.sha256()
    for f in ("rg_brick.hip", "rg_brick.hpp", "rg_math.hpp", "rg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2607_20704_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
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


def _median(xs):
    ys = sorted(xs)
    n = len(ys)
    return ys[n // 2] if n % 2 else 0.5 * (ys[n // 2 - 1] + ys[n // 2])


def time_form(D, u0, w, form, steps, warmup, api, tune=None, reps=5):
    """Timed steps on tree D: `reps` repetitions of exactly `steps` steps,
    each bracketed by device synchronisations; the median repetition is
    reported.  The time step of each step is folded into the previous
    step's update (cells no correction touches) and the corrected coarse
    cells' pass, as rg_step does with RG_STEP_CHAIN_DT; the first one comes
    from the separate CFL pass, outside the timed region."""
    import torch
    a, b = u0.clone(), torch.empty_like(u0)
    n = warmup + 2 * reps * steps + 1
    dts = torch.empty(n, dtype=torch.float64, device="cuda")
    api.cfl_dt(a, D.son_mask, D.level_begin, D.lmin, D.lmax, w.gamma, w.cfl, dts[0:1])
    # each step rebuilds the FNV hash and the neighbour lists from the keys;
    # re-keying (encode + radix sort + level ranges, only needed when the tree
    # changes) is timed on its own below
    flags = api.RG_STEP_REBUILD
    k = [0]

    def one_step(a, b, h0=None, h1=None, prepare=True):
        s = k[0]
        dt, dt_next = dts[s:s + 1], dts[s + 1:s + 2]
        if prepare:
            D.prepare(flags)
        dt_next.fill_(float("inf"))
        if h0 is not None:
            h0.record()
        for l in range(D.lmin, D.lmax + 1):
            D.hydro_level(l, dt, w.gamma, a, b, form, tune, w.cfl, dt_next)
        if h1 is not None:
            h1.record()
        if D.lmax > D.lmin:
            api.apply_coarse_corrections(b, D.corr, D.corr_base, D.nbr27, D.corr_base, D.n)
            api.cfl_dt_corrected(b, D.nbr27, D.level_begin, D.lmin, D.lmax, w.gamma, w.cfl, dt_next)
            for l in range(D.lmax, D.lmin, -1):
                api.restrict_level(b, D.father_cell, int(D.level_begin[l]), int(D.level_begin[l + 1]))
        k[0] = s + 1

    def ev():
        return torch.cuda.Event(enable_timing=True)

    for _ in range(warmup):
        one_step(a, b)
        a, b = b, a
    rep_ms, rep_hydro, rep_wall = [], [], []
    for _ in range(reps):
        h0 = [ev() for _ in range(steps)]
        h1 = [ev() for _ in range(steps)]
        start, end = ev(), ev()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        for i in range(steps):
            one_step(a, b, h0[i], h1[i])
            a, b = b, a
        end.record()
        torch.cuda.synchronize()
        rep_wall.append(1e3 * (time.perf_counter() - t0) / steps)
        rep_ms.append(start.elapsed_time(end) / steps)
        rep_hydro.append(sum(x.elapsed_time(y) for x, y in zip(h0, h1)) / steps)
    # hydro-only steps (dt + update with prebuilt lists), for the paper's
    # "Godunov solver only" comparison
    rep_only = []
    for _ in range(reps):
        s2, e2 = ev(), ev()
        torch.cuda.synchronize()
        s2.record()
        for i in range(steps):
            one_step(a, b, prepare=False)
            a, b = b, a
        e2.record()
        torch.cuda.synchronize()
        rep_only.append(s2.elapsed_time(e2) / steps)
    s3, e3 = ev(), ev()
    s3.record()
    for i in range(steps):
        D.prepare(api.L.RG_STEP_REKEY)
    e3.record()
    torch.cuda.synchronize()
    rekey_ms = s3.elapsed_time(e3) / steps
    # the folded time steps are the separate pass's, bit for bit
    check = api.cfl_dt(a, D.son_mask, D.level_begin, D.lmin, D.lmax, w.gamma, w.cfl)
    if float(check.cpu()[0]) != float(dts[k[0]].cpu()):
        raise RuntimeError("folded time step differs from the CFL pass")
    return {"ms_per_step": _median(rep_ms), "reps_ms_per_step": [round(x, 4) for x in rep_ms],
            "wall_ms_per_step": _median(rep_wall), "hydro_kernel_ms": _median(rep_hydro),
            "hydro_only_ms_per_step": _median(rep_only), "rekey_ms": rekey_ms, "state": a}


def device_check_run(D, u0, w, form, nsteps, tune):
    """`nsteps` steps from the initial state in the timed launch shape (hash
    and lists rebuilt every step, each dt folded into the previous update),
    for the parity re-check against the oracle; host copies."""
    import torch
    u, dts = D.run(u0, w.gamma, w.cfl, nsteps, form=form, rebuild=True, tune=tune, chain=True)
    torch.cuda.synchronize()
    return u.cpu().numpy(), dts.cpu().numpy()


def time_batched(forms, nsteps, reps, api, inputs, autotune):
    """The batched workload: 64 seeded boxes of uneven size and depth, all
    advanced `nsteps` steps by one graph launch; against the same boxes
    stepped one after another with rg_step (same kernels, one tree at a
    time)."""
    import torch
    boxes = inputs.batched_boxes(nbox=64, seed=20704, nsteps=nsteps)
    trees = [api.DeviceTree(b.ijkl, b.bc) for b in boxes]
    states = [D.to_key_order(b.u.reshape(-1, 5)) for D, b in zip(trees, boxes)]
    torch.cuda.synchronize()
    cells = sum(8 * D.n for D in trees)
    gammas, cfls = [b.gamma for b in boxes], [b.cfl for b in boxes]
    out = {"workload": "64 boxes, seed 20704: base level 4-7, 0-2 extra levels on a random sphere, Sod/Sedov/random "
                       "initial states; %d steps per box, one graph launch" % nsteps,
           "boxes": len(boxes), "cells": cells, "octs": sum(D.n for D in trees)}
    for f in forms:
        form = api.RG_FP64 if f == "fp64" else api.RG_MIXED
        tune, _ = autotune.tune_batch(trees, states, gammas, cfls, form)
        B = api.Batch(trees, states, gammas, cfls, nsteps, form=form, tune=tune)
        B.run()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            B.run()
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        ms.sort()
        batched_ms = ms[len(ms) // 2]
        B.close()
        # the same boxes one after another
        us = [s.clone() for s in states]
        vs = [torch.empty_like(s) for s in states]
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k, D in enumerate(trees):
            x, y = us[k], vs[k]
            for _ in range(nsteps):
                D.step(x, y, gammas[k], cfls[k], form, dt=dt)
                x, y = y, x
        b.record()
        b.synchronize()
        seq_ms = a.elapsed_time(b)
        out[f] = {"cell_updates_per_s": cells * nsteps / (batched_ms * 1e-3),
                  "ms_per_launch": round(batched_ms, 3), "tune": list(tune),
                  "one_tree_at_a_time_cell_updates_per_s": cells * nsteps / (seq_ms * 1e-3)}
    return out


_DEEP = {}


def deep_workload(inputs):
    """The clumpy-gas deep tree, generated once per run (about a minute on
    the host)."""
    if "w" not in _DEEP:
        _DEEP["w"] = inputs.deep_amr()
    return _DEEP["w"]


def time_deep_amr(forms, nsteps, api, inputs, autotune=None, check_steps=0):
    """The clumpy-gas deep tree (base 7 up to level 12, about 28 M cells):
    `nsteps` whole steps per form (dt folded into the previous step's
    update as in the main workload, every level, corrections,
    restriction; lists prebuilt), and the mixed form's L1 error per
    conserved field against FP64 after those steps (leaf cells, volume
    weighted).  Also two coarse steps with level subcycling, reported as
    cell-updates/s and as simulated time advanced per wall second beside
    the global step's."""
    import numpy as np
    import torch
    w = deep_workload(inputs)
    D = api.DeviceTree(w.ijkl, w.bc)
    u0 = D.to_key_order(w.u)
    lv = torch.as_tensor(np.repeat(D.ijkl_sorted.cpu().numpy()[:, 3], 8), device="cuda")
    bits = torch.arange(8, device="cuda", dtype=torch.int32).repeat(D.n)
    leaf = ((D.son_mask.repeat_interleave(8) >> bits) & 1) == 0
    vol = torch.where(leaf, torch.pow(2.0, -3.0 * lv.double()), torch.zeros((), dtype=torch.float64, device="cuda"))
    cells = 8 * D.n
    out = {"workload": "clumpy gas, base level 7 refined cell by cell to level 12 where rho > 8 mean rho; 2000 "
                       "Gaussian clumps (seed 20705, lognormal amplitudes sigma %.4g), at rest, p = rho^(5/3), "
                       "gamma 5/3, periodic; %d steps" % (w.meta["sigma_a"], nsteps),
           "octs": D.n, "cells": cells,
           "octs_per_level": {str(l): int(D.level_begin[l + 1] - D.level_begin[l]) for l in range(D.lmin, D.lmax + 1)},
           "schedule": {str(l): {"bricks": c[0], "per_oct": c[1], "sibling_groups": c[2]} for l, c in D.schedule_counts().items()}}
    updates_sub = sum(2 ** (l - D.lmin) * 8 * int(D.level_begin[l + 1] - D.level_begin[l])
                      for l in range(D.lmin, D.lmax + 1))
    states, device = {}, {}
    for f in forms:
        form = api.RG_FP64 if f == "fp64" else api.RG_MIXED
        tune = autotune.tune_tree(D, u0, w.gamma, form)[0] if autotune else None
        D.run(u0, w.gamma, w.cfl, 1, form=form, tune=tune, chain=True)       # warm-up
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        u, dts = D.run(u0, w.gamma, w.cfl, nsteps, form=form, tune=tune, chain=True)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / nsteps
        states[f] = u
        out[f] = {"cell_updates_per_s": cells / (ms * 1e-3), "ms_per_step": round(ms, 4),
                  "tune": list(tune) if tune else None}
        if check_steps:
            device[f] = device_check_run(D, u0, w, form, check_steps, tune)
        global_dt = float(dts.mean())
        # the same steps with the sibling groups left to the per-oct kernel
        base = list(tune[:5]) if tune else [4, 256, 0, 0, 0]
        ng = tuple(base + [0] * (5 - len(base)) + [1, 0])
        D.run(u0, w.gamma, w.cfl, 1, form=form, tune=ng, chain=True)
        a.record()
        D.run(u0, w.gamma, w.cfl, nsteps, form=form, tune=ng, chain=True)
        b.record()
        b.synchronize()
        out[f]["ms_per_step_without_sibling_groups"] = round(a.elapsed_time(b) / nsteps, 4)
        # level subcycling: level l takes 2^(l - lmin) steps per coarse step
        nsub = 2
        D.run_subcycled(u0, w.gamma, w.cfl, 1, form=form, tune=tune)     # warm-up
        torch.cuda.synchronize()
        a.record()
        _, sdts = D.run_subcycled(u0, w.gamma, w.cfl, nsub, form=form, tune=tune)
        b.record()
        b.synchronize()
        sms = a.elapsed_time(b) / nsub
        sdt = float(sdts.mean())
        out[f]["subcycled"] = {
            "ms_per_coarse_step": round(sms, 3), "coarse_steps": nsub,
            "cell_updates_per_coarse_step": updates_sub,
            "cell_updates_per_s": updates_sub / (sms * 1e-3),
            "coarse_dt": sdt, "global_dt": global_dt,
            "simulated_time_per_s": sdt / (sms * 1e-3),
            "global_simulated_time_per_s": global_dt / (ms * 1e-3),
        }
    # coarse ghost cells by linear interpolation (the per-oct kernel's second
    # instantiation; bricks have no coarse ghosts)
    if "fp64" in forms:
        tune = out["fp64"]["tune"]
        DL = api.DeviceTree(w.ijkl, w.bc, ghost=api.L.RG_GHOST_LINEAR)
        DL.run(u0, w.gamma, w.cfl, 1, form=api.RG_FP64, tune=tune, chain=True)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        DL.run(u0, w.gamma, w.cfl, nsteps, form=api.RG_FP64, tune=tune, chain=True)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / nsteps
        out["fp64"]["linear_ghosts"] = {"ms_per_step": round(ms, 4), "cell_updates_per_s": cells / (ms * 1e-3)}
        del DL
    if "fp64" in states and "mixed" in states:
        x, y = states["fp64"], states["mixed"]
        num = (vol[:, None] * (x - y).abs()).sum(0)
        den = (vol[:, None] * x.abs()).sum(0)
        rho_den = den[0]
        l1 = [float(num[0] / den[0])] + [float(num[v] / rho_den) for v in (1, 2, 3)] + [float(num[4] / den[4])]
        out["mixed"]["l1_vs_fp64_after_%d_steps" % nsteps] = l1
        out["mixed"]["l1_note"] = "momenta start at rest: their L1 is relative to the density norm"
    return out, device


def time_sedov(forms, steps, warmup, api, inputs, autotune=None, check_steps=0):
    """The Sedov blast on its graded AMR tree (base level 6, refined to level
    8 inside r < 0.15 of the centre): whole global steps per form, timed like
    the main workload (hash and lists rebuilt, dt folded, corrections,
    corrected cells' dt, restriction; median of 5 repetitions).  Returns the
    report, the workload and, with check_steps, each form's state after
    that many steps from the initial state (host copies)."""
    w = inputs.sedov_amr()
    D = api.DeviceTree(w.ijkl, w.bc)
    u0 = D.to_key_order(w.u)
    cells = 8 * D.n
    out = {"workload": "Sedov blast: base level 6 (64^3) refined to level 8 inside r < 0.15 of the centre, rho 1, "
                       "p 1e-5, E 1 in the central cell, gamma 1.4, periodic, CFL 0.8; %d global steps" % steps,
           "octs": D.n, "cells": cells, "levels": [D.lmin, D.lmax],
           "octs_per_level": {str(l): int(D.level_begin[l + 1] - D.level_begin[l]) for l in range(D.lmin, D.lmax + 1)},
           "schedule": {str(l): {"bricks": c[0], "per_oct": c[1], "sibling_groups": c[2]}
                        for l, c in D.schedule_counts().items()}}
    device = {}
    for f in forms:
        form = api.RG_FP64 if f == "fp64" else api.RG_MIXED
        tune = autotune.tune_tree(D, u0, w.gamma, form)[0] if autotune else None
        r = time_form(D, u0, w, form, steps, warmup, api, tune)
        out[f] = {"cell_updates_per_s": cells / (r["ms_per_step"] * 1e-3), "ms_per_step": round(r["ms_per_step"], 4),
                  "reps_ms_per_step": r["reps_ms_per_step"],
                  "hydro_only_cell_updates_per_s": cells / (r["hydro_only_ms_per_step"] * 1e-3),
                  "hydro_kernels_ms_per_step": round(r["hydro_kernel_ms"], 4),
                  "tune": list(tune) if tune else None}
        if check_steps:
            device[f] = device_check_run(D, u0, w, form, check_steps, tune)
    return out, w, device


def time_dynamic(api, inputs):
    """Tree changes on the device (refinement, de-refinement, sort, hash and
    neighbour rebuild: rg_refine; kernel schedule: rg_schedule_build_device).
    Deep AMR: refinement passes with the criterion the tree was built with
    (rho > 8 mean rho, finest level 12) beside one FP64 hydro step of the
    same tree.  Sedov (base 6, up to level 8): every step a hydro step, then
    refinement on the density jump (> 0.08), then the schedule; wall time per
    step with its parts."""
    import torch

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    out = {}
    w = deep_workload(inputs)
    n = len(w.ijkl)
    D = api.DeviceTree(w.ijkl, w.bc, capacity=int(1.25 * n))
    thr = 8.0 * w.meta["mean_rho"]
    bufs = [D.to_key_order(w.u), torch.empty((8 * D.capacity, 5), dtype=torch.float64, device="cuda")]
    full = torch.empty((8 * D.capacity, 5), dtype=torch.float64, device="cuda")
    full[:8 * D.n] = bufs[0]
    bufs[0] = full
    cur = 0
    refine_ms, sched_ms, octs = [], [], []
    for it in range(4):
        _, ms = wall(lambda: D.refine(bufs[cur][:8 * D.n], thr, 0.0, 12, out=bufs[cur ^ 1], schedule=False))
        cur ^= 1
        _, ms2 = wall(lambda: D.build_schedule())
        if it:
            refine_ms.append(ms)
            sched_ms.append(ms2)
        octs.append(D.n)
    _, host_sched_ms = wall(lambda: D.build_schedule(on_host=True))
    D.build_schedule()
    u = bufs[cur][:8 * D.n]
    a = torch.empty_like(u)
    D.step(u, a, w.gamma, w.cfl, api.RG_FP64)
    _, step_ms = wall(lambda: D.step(u, a, w.gamma, w.cfl, api.RG_FP64))
    out["deep_amr_refine"] = {
        "octs_per_pass": octs, "refine_ms": round(min(refine_ms), 3), "schedule_ms": round(min(sched_ms), 3),
        "host_schedule_ms": round(host_sched_ms, 1), "hydro_step_ms": round(step_ms, 3),
        "note": "refine = flags, closure, new oct list, key sort, state gather, level ranges, hash, neighbours"}
    del bufs, full, u, a, D
    torch.cuda.empty_cache()

    def sedov(nsubgrid):
        w = inputs.sedov_amr()
        D = api.DeviceTree(w.ijkl, w.bc, capacity=400000)
        u = torch.empty((8 * D.capacity, 5), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        u[:8 * D.n] = D.to_key_order(w.u)
        parts = {"step": 0.0, "refine": 0.0, "schedule": 0.0}
        cells = 0
        nsteps, warm = 20, 5
        for s in range(warm + nsteps):
            n8 = 8 * D.n
            _, t1 = wall(lambda: D.step(u[:n8], v[:n8], w.gamma, w.cfl, api.RG_FP64))
            _, t2 = wall(lambda: D.refine(v[:n8], 0.0, 0.08, 8, out=u, schedule=False, nsubgrid=nsubgrid))
            _, t3 = wall(lambda: D.build_schedule())
            if s >= warm:
                parts["step"] += t1
                parts["refine"] += t2
                parts["schedule"] += t3
                cells += n8
        total = sum(parts.values())
        return {
            "workload": "Sedov blast, base level 6, refined on |rho_n - rho| / (rho_n + rho) > 0.08 up to level 8, "
                        "FP64, refinement every step, nsubgrid %d" % nsubgrid,
            "steps": nsteps, "octs_at_end": D.n,
            "bricks_at_end": sum(c[0] for c in D.schedule_counts().values()),
            "ms_per_step": round(total / nsteps, 3),
            "parts_ms_per_step": {k: round(v_ / nsteps, 3) for k, v_ in parts.items()},
            "cell_updates_per_s": cells / (total * 1e-3)}

    # the Sedov configuration's tree (67 k octs), subcycled: launched step by
    # step, and captured once as a HIP graph and replayed
    w = inputs.sedov_amr()
    D = api.DeviceTree(w.ijkl, w.bc)
    u = D.to_key_order(w.u)
    nrep = 20
    for _ in range(2):
        D.step_subcycled(u, w.gamma, w.cfl)
    _, eager_ms = wall(lambda: [D.step_subcycled(u, w.gamma, w.cfl) for _ in range(nrep)])
    g = D.capture_subcycled(u, w.gamma, w.cfl)
    g.replay()
    _, graph_ms = wall(lambda: [g.replay() for _ in range(nrep)])
    ups = sum(2 ** (l - D.lmin) * 8 * int(D.level_begin[l + 1] - D.level_begin[l]) for l in range(D.lmin, D.lmax + 1))
    out["sedov_subcycled"] = {
        "workload": "Sedov blast tree, base 6 to level 8 (67,344 octs), FP64 subcycled coarse steps",
        "cell_updates_per_coarse_step": ups,
        "launched_ms_per_coarse_step": round(eager_ms / nrep, 4),
        "graph_ms_per_coarse_step": round(graph_ms / nrep, 4),
        "graph_cell_updates_per_s": ups / (graph_ms / nrep * 1e-3)}
    del g, D, u
    out["sedov_dynamic"] = sedov(2)
    out["sedov_dynamic_blocks"] = sedov(4)
    return out


def time_mg(api, level=8, ncycles=5):
    """Multigrid Poisson V-cycles (Sec. 5) on the periodic level-`level`
    unigrid (256^3 by default): Lap phi = f with a seeded zero-mean random
    f, 2 + 2 red-black sweeps per level, down to level 1 with 50 sweeps
    there.  Reports cell-updates per second per V-cycle (fine cells over the
    cycle's time, the paper's unit) and the residual reduction per cycle."""
    import numpy as np
    import torch
    M = api.Multigrid(level)
    N = 1 << level
    rng = np.random.default_rng(20704)
    f = rng.standard_normal(N ** 3)
    f -= f.mean()
    M.f[M.fine] = torch.as_tensor(f).cuda()
    r0 = float(torch.sqrt((M.residual() ** 2).mean()))
    M.vcycles(1)
    r1 = float(torch.sqrt((M.residual() ** 2).mean()))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    M.vcycles(ncycles)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / ncycles
    r2 = float(torch.sqrt((M.residual() ** 2).mean()))
    cells = N ** 3
    return {"workload": "Poisson Lap phi = f on a %d^3 periodic unigrid, seeded zero-mean random f, V(2,2) cycles "
                        "to level 1" % N,
            "ms_per_vcycle": round(ms, 4), "cell_updates_per_s_per_vcycle": cells / (ms * 1e-3),
            "residual_rms": [r0, r1, r2], "residual_factor_per_cycle": (r2 / r1) ** (1.0 / ncycles),
            "octs_in_hierarchy": M.tree.n}


def time_mg_amr(api, inputs, trees=("sedov", "deep"), ncycles=4, reps=5):
    """The level-by-level multigrid on AMR trees (rg_mg_level_*): per level,
    the hierarchy build, the time of one V-cycle (median of `reps`), the
    level's cell-updates per second per V-cycle and the residual factor per
    cycle over `ncycles` cycles from zero; then the whole solve (every level
    in turn, `ncycles` cycles each).  Random right-hand side (zero mean on
    the coarsest level), seed 20704."""
    import numpy as np
    import torch
    out = {}
    for name in trees:
        w = inputs.sedov_amr() if name == "sedov" else deep_workload(inputs)
        D = api.DeviceTree(w.ijkl, w.bc)
        rng = np.random.default_rng(20704)
        f = rng.standard_normal(8 * D.n)
        cb, ce = 8 * int(D.level_begin[D.lmin]), 8 * int(D.level_begin[D.lmin + 1])
        f[cb:ce] -= f[cb:ce].mean()
        fd = torch.as_tensor(f, device="cuda")
        phi = torch.zeros_like(fd)
        r = torch.zeros_like(fd)
        levels = {}
        total_ms = 0.0
        for l in range(D.lmin, D.lmax + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = api.MgLevel(D, l)
            build_ms = 1e3 * (time.perf_counter() - t0)
            res = []
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(ncycles)]
            for c in range(ncycles):
                ev[c][0].record()
                h.vcycles(phi, fd, 1)
                ev[c][1].record()
                rr = h.residual(phi, fd, r)
                res.append(float(torch.sqrt((rr * rr).mean())))
            torch.cuda.synchronize()
            total_ms += sum(a.elapsed_time(b) for a, b in ev)
            # timing: further cycles from the converged state (same work)
            times = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                h.vcycles(phi, fd, 1)
                b.record()
                b.synchronize()
                times.append(a.elapsed_time(b))
            ms = _median(times)
            cells = 8 * int(D.level_begin[l + 1] - D.level_begin[l])
            levels[str(l)] = {"cells": cells, "hierarchy_octs": h.counts(), "build_ms": round(build_ms, 3),
                              "ms_per_vcycle": round(ms, 4), "cell_updates_per_s_per_vcycle": cells / (ms * 1e-3),
                              "residual_rms": res,
                              "residual_factor_per_cycle": (res[-1] / res[0]) ** (1.0 / max(1, ncycles - 1))}
            h.close()
        cells_all = 8 * D.n
        out[name] = {"workload": ("Sedov blast tree (base 6, refined to 8 inside r < 0.15)" if name == "sedov" else
                                  "clumpy-gas deep tree (base 7 to level 12)") +
                     ", Lap phi = f with a seeded random f, V(2,2) cycles to level 1, each level solved in turn "
                     "with the coarser potential as boundary values",
                     "octs": D.n, "levels": levels,
                     "solve_ms_%d_cycles_per_level" % ncycles: round(total_ms, 3),
                     "cell_updates_per_s_per_vcycle": cells_all * ncycles / (total_ms * 1e-3)}
        del D, fd, phi, r
        torch.cuda.empty_cache()
    return out


def copy_ceiling(torch, mib=1024, reps=5):
    """Practical HBM ceiling: GB/s (read + write) of a plain device copy of
    `mib` MiB, best of `reps`."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * n * 8 / (best * 1e-3) / 1e9


FP64_BAR = 1e-12
MIXED_L1_BAR = 1e-5


def _parity_ratio(got, ref):
    """Worst per-cell ratio of the FP64 bar: |d| / |ref| for density and
    energy, |d| / max|ref| for each momentum component (<= 1e-12 passes)."""
    import numpy as np
    d = np.abs(got - ref)
    worst = 0.0
    for v in range(5):
        scale = np.abs(ref[:, v]) if v in (0, 4) else np.full(len(ref), np.abs(ref[:, v]).max())
        ok = scale > 0
        r = np.where(ok, d[:, v] / np.where(ok, scale, 1.0), np.where(d[:, v] > 0, np.inf, 0.0))
        worst = max(worst, float(r.max()))
    return worst


def _mixed_l1(got, ref, T):
    """Per conserved field: sum V |x - x_ref| / sum V |x_ref| over leaf cells;
    momenta against the larger of their own norm and the density norm (a
    field that starts at rest has no norm of its own)."""
    import numpy as np
    leaf = (((T.son_mask[:, None] >> np.arange(8)[None, :]) & 1) == 0).reshape(-1)
    vol = np.repeat((0.5 ** T.ijkl[:, 3].astype(np.float64)) ** 3, 8) * leaf
    num = (vol[:, None] * np.abs(got - ref)).sum(0)
    den = (vol[:, None] * np.abs(ref)).sum(0)
    den[1:4] = np.maximum(den[1:4], den[0])
    return [float(x) for x in num / den]


def cpu_baseline(cases, sample_octs):
    """The oracle, as it stands, on the host, and the in-run parity re-check.

    cases: name -> (workload, omp_steps, serial, device) with serial either
    ("steps", n) (whole steps of the serial oracle) or ("octs", ob, oe) (the
    serial oracle's hydro update of octs [ob, oe), with the first step's
    dt), and device a dict form -> (state, dts) of the device after
    omp_steps steps from the same initial state.  Per case the OpenMP build
    of the oracle runs omp_steps whole steps on every host core; its state
    is the expected value of the device's, FP64 per cell within 1e-12 (and
    the time steps), the mixed form's L1 per field within 1e-5."""
    import numpy as np

    from oracle import oracle as O
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    configs, parity, ok = {}, {}, True
    for name, (w, omp_steps, serial, device) in cases.items():
        log("oracle: %s" % name)
        T = O.Tree(w.ijkl, w.bc)
        u = T.permute_cells(w.u)
        cells = 8 * T.n
        ref = u.copy()
        with O.threads():
            threads = O.nthreads()
            t0 = time.perf_counter()
            ref_dts = T.run(ref, w.gamma, w.cfl, omp_steps)
            sec = time.perf_counter() - t0
        c = {"octs": T.n, "cells": cells,
             "omp": {"value": cells * omp_steps / sec, "cores": threads, "steps": omp_steps, "seconds": round(sec, 2)}}
        if serial[0] == "steps":
            x = u.copy()
            t0 = time.perf_counter()
            T.run(x, w.gamma, w.cfl, serial[1])
            sec1 = time.perf_counter() - t0
            c["serial"] = {"value": cells * serial[1] / sec1, "cores": 1, "steps": serial[1],
                           "seconds": round(sec1, 2)}
        else:
            ob, oe = serial[1], min(serial[2], T.n)
            unew = np.zeros_like(u)
            corr = np.zeros(1)
            t0 = time.perf_counter()
            O.hydro_octs(T.ijkl, T.nbr27, T.son_mask, ob, oe, u, unew, corr, float(ref_dts[0]), w.gamma)
            sec1 = time.perf_counter() - t0
            c["serial"] = {"value": 8 * (oe - ob) / sec1, "cores": 1, "octs": [ob, oe],
                           "what": "hydro update of octs [%d, %d) (first step's dt)" % (ob, oe),
                           "seconds": round(sec1, 2)}
        configs[name] = c
        p = {"steps": omp_steps}
        if "fp64" in device:
            got, dts = device["fp64"]
            p["fp64_worst_ratio"] = _parity_ratio(got, ref)
            p["fp64_dt_worst_rel"] = float(np.max(np.abs(dts - ref_dts) / ref_dts))
            good = p["fp64_worst_ratio"] <= FP64_BAR and p["fp64_dt_worst_rel"] <= FP64_BAR
            p["fp64_ok"] = bool(good)
            ok = ok and good
        if "mixed" in device:
            got, _ = device["mixed"]
            p["mixed_l1"] = _mixed_l1(got, ref, T)
            good = max(p["mixed_l1"]) <= MIXED_L1_BAR
            p["mixed_ok"] = bool(good)
            ok = ok and good
        parity[name] = p
        log("  oracle %d threads %.1f s, serial %.1f s; parity %s" % (threads, sec, sec1, p))
        del T, u, ref
    hname = "random256" if "random256" in configs else next(iter(configs))
    head = configs[hname]
    what = "the same 256^3 box" if hname == "random256" else "the %s workload" % hname
    base = {"value": head["omp"]["value"], "unit": "cell-updates/s", "cores": head["omp"]["cores"], "kind": "oracle",
            "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
            "sample": "%d whole step(s) of %s (CFL dt, neighbour lists prebuilt, hydro update of every oct, "
                      "corrections, restriction) by the oracle's OpenMP build on %d threads, %.1f s"
                      % (head["omp"]["steps"], what, head["omp"]["cores"], head["omp"]["seconds"]),
            "serial": {"value": head["serial"]["value"], "cores": 1,
                       "sample": "%s of %s, serial FP64 oracle, %.1f s"
                                 % (head["serial"].get("what", "%d whole step(s)" % head["serial"].get("steps", 0)),
                                    what, head["serial"]["seconds"])},
            "configs": configs}
    return base, {"ok": bool(ok), "fp64_bar": FP64_BAR, "mixed_l1_bar": MIXED_L1_BAR, "cases": parity,
                  "note": "device state after the same steps from the same initial state, in the timed launch shape "
                          "(hash and lists rebuilt, dt folded), against the oracle's OpenMP build"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-octs", type=int, default=1 << 19,
                    help="octs of the 256^3 box in the serial oracle's timed update")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-box batched workload")
    ap.add_argument("--no-tune", action="store_true", help="library default kernels instead of autotuned ones")
    ap.add_argument("--no-deep-amr", action="store_true", help="skip the clumpy-gas deep-AMR workload")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the refinement (dynamic tree) measurements")
    ap.add_argument("--no-mg", action="store_true", help="skip the multigrid Poisson measurement")
    ap.add_argument("--no-sedov", action="store_true", help="skip the Sedov AMR global-step workload")
    ap.add_argument("--leg", choices=["all", "deep_amr", "dynamic", "mg_poisson", "mg_amr"], default="all",
                    help="run one workload only and print its JSON (for profiling it); 'all' is the benchmark line")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d requested)" % args.gpus)

    import numpy as np
    import torch

    from paper_2607_20704_amd import api, autotune, inputs
    torch.cuda.set_device(0)
    if args.leg != "all":
        forms = [f.strip() for f in args.forms.split(",") if f.strip()]
        leg = (time_deep_amr(forms, 10, api, inputs, None if args.no_tune else autotune)[0] if args.leg == "deep_amr" else
               time_dynamic(api, inputs) if args.leg == "dynamic" else
               time_mg_amr(api, inputs) if args.leg == "mg_amr" else time_mg(api))
        print(json.dumps({args.leg: leg}), flush=True)
        return
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
    copy_gbs = copy_ceiling(torch)
    log("plain device copy: %.0f GB/s" % copy_gbs)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    res = {}
    for f in forms:
        form = api.RG_FP64 if f == "fp64" else api.RG_MIXED
        tune = None
        if not args.no_tune:
            tune, times = autotune.tune_tree(D, u0, w.gamma, form)
            log("form %s: autotuned %s" % (f, tune))
            for c, t in sorted(times.items(), key=lambda kv: kv[1]):
                log("    %-24s %.4f ms" % (c, t))
        log("timing form %s: %d warmup + %d steps" % (f, args.warmup, args.steps))
        res[f] = time_form(D, u0, w, form, args.steps, args.warmup, api, tune, REPS)
        res[f]["tune"] = list(tune) if tune else None
        log("  %.3f ms/step, hydro kernel %.3f ms" % (res[f]["ms_per_step"], res[f]["hydro_kernel_ms"]))

    def roof(r, f):
        achieved = ALG_BYTES_PER_CELL * cells / (r["hydro_kernel_ms"] * 1e-3) / 1e9
        # the box is a complete periodic level: its bricks go two by two
        # along z unless the chosen variant turns that off
        single = r["tune"] is not None and len(r["tune"]) > 7 and r["tune"][7]
        kernel = "k_hydro_brick" if single else "k_hydro_brick_pair"
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f),
                "copy_ceiling": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "kernel": kernel, "alg_bytes_per_launch": ALG_BYTES_PER_CELL * cells,
                "kernel_ms": round(r["hydro_kernel_ms"], 4)}

    def summary(r, f):
        return {"value": cells / (r["ms_per_step"] * 1e-3), "ms_per_step": round(r["ms_per_step"], 4),
                "hydro_only_cell_updates_per_s": cells / (r["hydro_only_ms_per_step"] * 1e-3),
                "hydro_only_ms_per_step": round(r["hydro_only_ms_per_step"], 4),
                "rekey_ms": round(r["rekey_ms"], 4),
                "ns_per_cell": r["ms_per_step"] * 1e6 / cells, "tune": r["tune"], "roofline": roof(r, f)}

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
                     "schedule": {str(l): {"bricks": c[0], "per_oct": c[1], "sibling_groups": c[2]} for l, c in D.schedule_counts().items()},
                     "step": "hash rebuild + neighbour lists + hydro with the next dt folded in (+ corrections "
                             "+ corrected cells' dt + restriction)"}
    out["roofline"] = s["roofline"]
    out["hydro_only_cell_updates_per_s"] = s["hydro_only_cell_updates_per_s"]
    out["rekey_ms"] = s["rekey_ms"]
    out["tune"] = s["tune"]
    out["ns_per_cell"] = s["ns_per_cell"]
    for f in forms:
        if f != primary:
            out[f] = summary(res[f], f)
            out[f]["dtype"] = "f32-flux/f64-state" if f == "mixed" else "f64"
    if "fp64" in res and "mixed" in res:
        a, b = res["fp64"]["state"], res["mixed"]["state"]
        l1 = ((a - b).abs().sum(0) / a.abs().sum(0).clamp_min(1e-300)).cpu().numpy()
        out["mixed"]["l1_vs_fp64_after_%d_steps" % (2 * REPS * args.steps + args.warmup)] = [float(x) for x in l1]
    out["reps"] = REPS
    out["reps_ms_per_step"] = res[primary]["reps_ms_per_step"]
    # the parity re-check: states after a few steps from the initial state, in
    # the timed launch shape, compared with the oracle in the CPU leg below
    cases = {}
    if not args.no_cpu_baseline:
        log("parity re-check runs: 256^3 box, 1 step")
        dev = {f: device_check_run(D, u0, w, api.RG_FP64 if f == "fp64" else api.RG_MIXED, 1, res[f]["tune"])
               for f in forms}
        cases["random256"] = (w, 1, ("octs", 0, args.cpu_sample_octs), dev)
        log("parity re-check runs: Sod tube, 20 steps")
        ws = inputs.sod_uniform()
        Ds = api.DeviceTree(ws.ijkl, ws.bc)
        cases["sod_l5"] = (ws, 20, ("steps", 20),
                           {"fp64": device_check_run(Ds, Ds.to_key_order(ws.u), ws, api.RG_FP64, 20, None)})
        del Ds
    if not args.no_sedov:
        log("Sedov AMR global steps")
        out["sedov_amr"], wsd, dev = time_sedov(forms, args.steps, args.warmup, api, inputs,
                                                None if args.no_tune else autotune,
                                                0 if args.no_cpu_baseline else 20)
        if dev:
            cases["sedov_amr"] = (wsd, 20, ("steps", 2), dev)
        torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched workload")
        del res
        torch.cuda.empty_cache()
        out["batched"] = time_batched(forms, 20, 5, api, inputs, autotune)
        torch.cuda.empty_cache()
    if not args.no_deep_amr:
        log("deep-AMR workload: generating")
        out["deep_amr"], dev = time_deep_amr(forms, 10, api, inputs, None if args.no_tune else autotune,
                                             0 if args.no_cpu_baseline else 1)
        if dev:
            cases["deep_amr"] = (deep_workload(inputs), 1, ("octs", 0, 1 << 17), dev)
        torch.cuda.empty_cache()
    if not args.no_mg:
        log("multigrid Poisson V-cycles")
        out["mg_poisson"] = time_mg(api)
        torch.cuda.empty_cache()
        log("multigrid on the AMR trees, level by level")
        out["mg_poisson_amr"] = time_mg_amr(api, inputs, ("sedov",) if args.no_deep_amr else ("sedov", "deep"))
        torch.cuda.empty_cache()
    if not args.no_dynamic:
        log("dynamic trees: refinement on the device")
        out["dynamic"] = time_dynamic(api, inputs)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("oracle on the host: timings and the parity re-check")
        order = ["sod_l5", "sedov_amr", "random256", "deep_amr"]
        out["cpu_baseline"], out["parity"] = cpu_baseline({k: cases[k] for k in order if k in cases},
                                                          args.cpu_sample_octs)
        if not out["parity"]["ok"]:
            out["value"] = None
            print(json.dumps(out), flush=True)
            sys.exit("the device state differs from the oracle's beyond the stated bars")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
