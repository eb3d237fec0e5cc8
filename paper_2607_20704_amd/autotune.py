"""Kernel-variant selection by measurement.

Every variant the library offers for a workload (octs per workgroup of the
per-oct kernel, bricks on or off, sibling groups on or off and their
workgroup size, the brick kernel's register budget, persistent or
one-item-per-workgroup batched grids) computes the same bits -- the GPU
tests check this -- so the choice only changes speed.  The tuner times each candidate with HIP events
on the caller's device and keeps the fastest in a JSON cache keyed by device
name, form and a coarse workload signature, so later runs reuse it.

The cache file is $RG_TUNE_CACHE, else ~/.cache/rg_tune.json; set
RG_TUNE_CACHE=off to measure every time without reading or writing a file.
"""
import json
import math
import os

import torch

from . import api

# (octs_per_group, threads, no_bricks, persistent, brick_waves, no_groups,
# group_threads, no_pairs): per-oct workgroup shapes, bricks off, sibling
# groups off or on other workgroup sizes, bricks one by one where they could
# go in pairs, and the brick kernel's register budgets
TREE_CANDIDATES = [(4, 256, 0, 0, 0), (2, 128, 0, 0, 0), (8, 256, 0, 0, 0), (7, 256, 0, 0, 0), (3, 128, 0, 0, 0),
                   (4, 256, 1, 0, 0), (4, 256, 0, 0, 0, 1, 0), (4, 256, 0, 0, 0, 0, 256), (4, 256, 0, 0, 0, 0, 384),
                   (4, 256, 0, 0, 0, 0, 0, 1)]
BRICK_WAVES = {api.RG_FP64: (2, 3), api.RG_MIXED: (3, 4)}


def tree_candidates(form):
    out = list(TREE_CANDIDATES)
    for w in BRICK_WAVES[form]:
        out.append((4, 256, 0, 0, w))
    return out


# (octs_per_group, threads, no_bricks, persistent[, brick_waves, no_groups])
BATCH_CANDIDATES = ([(g, 256, nb, p) for g in (2, 4, 8) for nb in (0, 1) for p in (0, 1)] +
                    [(g, 256, 0, p, 0, 1) for g in (2, 4, 8) for p in (0, 1)])


def _cache_path():
    p = os.environ.get("RG_TUNE_CACHE")
    if p == "off":
        return None
    return p or os.path.join(os.path.expanduser("~"), ".cache", "rg_tune.json")


def _load():
    p = _cache_path()
    if not p or not os.path.exists(p):
        return {}
    try:
        with open(p) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    p = _cache_path()
    if not p:
        return
    d = _load()
    d[key] = value
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _device():
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace(" ", "_")


def _bucket(n):
    return int(round(math.log2(max(int(n), 1))))


def _time(fn, reps):
    """Median of `reps` event-timed calls of fn (after one untimed call)."""
    fn()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tree_signature(D):
    counts = D.schedule_counts().values()
    bricks = sum(c[0] for c in counts)
    groups = sum(c[2] for c in counts)
    return "n%d_l%d-%d_b%d_g%d" % (_bucket(D.n), D.lmin, D.lmax, _bucket(512 * bricks + 1), _bucket(8 * groups + 1))


def tune_tree(D, u, gamma, form, reps=5, use_cache=True, candidates=None):
    """Fastest tuning for the update of every level of tree D (state u, key
    order).  Returns (tuning tuple, {candidate: ms})."""
    key = "tree|%s|%s|%s" % (_device(), "fp64" if form == api.RG_FP64 else "mixed", tree_signature(D))
    if use_cache:
        hit = _load().get(key)
        if hit:
            return tuple(hit["best"]), {}
    candidates = candidates or tree_candidates(form)
    dt = api.cfl_dt(u, D.son_mask, D.level_begin, D.lmin, D.lmax, gamma, 0.8)
    out = torch.empty_like(u)
    times = {}
    for c in candidates:
        def run(c=c):
            for l in range(D.lmin, D.lmax + 1):
                D.hydro_level(l, dt, gamma, u, out, form, c)
        times[c] = _time(run, reps)
    best = min(times, key=times.get)
    _store(key, {"best": list(best), "ms": {str(k): v for k, v in times.items()}})
    return best, times


def batch_signature(trees):
    n = sum(D.n for D in trees)
    return "t%d_n%d_L%d" % (len(trees), _bucket(n), max(D.lmax for D in trees))


def tune_batch(trees, states, gammas, cfls, form, nsteps=2, reps=3, use_cache=True, candidates=BATCH_CANDIDATES):
    """Fastest tuning of the batched form for these trees.  Each candidate
    is captured once (nsteps steps) and its graph launch timed.  Returns
    (tuning tuple, {candidate: ms per step})."""
    key = "batch|%s|%s|%s" % (_device(), "fp64" if form == api.RG_FP64 else "mixed", batch_signature(trees))
    if use_cache:
        hit = _load().get(key)
        if hit:
            return tuple(hit["best"]), {}
    times = {}
    for c in candidates:
        B = api.Batch(trees, states, gammas, cfls, nsteps, form=form, tune=c)
        times[c] = _time(B.run, reps) / nsteps
        B.close()
    best = min(times, key=times.get)
    _store(key, {"best": list(best), "ms_per_step": {str(k): v for k, v in times.items()}})
    return best, times
