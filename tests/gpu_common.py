"""Shared helpers of the GPU parity tests: build the same workload on the
device (through the C ABI) and in the oracle, and compare."""
import sys

import numpy as np

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def build_both(ijkl, bc):
    from paper_2607_20704_amd import api
    T = O.Tree(ijkl, bc)
    D = api.DeviceTree(ijkl, bc)
    keys = D.keys.cpu().numpy()
    assert np.array_equal(keys, T.keys), "device key order differs from the oracle's"
    return T, D


def parity_metric(got, ref):
    """Per-cell check of the FP64 bar: |d| <= tol |ref| for density and
    energy, |d| <= tol max|ref| for each momentum component.  Returns the
    worst ratio |d| / scale (so <= 1e-12 passes) and the max abs difference."""
    d = np.abs(got - ref)
    worst = 0.0
    for v in range(5):
        if v in (0, 4):
            scale = np.abs(ref[:, v])
        else:
            scale = np.full(len(ref), np.abs(ref[:, v]).max())
        ok = scale > 0
        r = np.where(ok, d[:, v] / np.where(ok, scale, 1.0), np.where(d[:, v] > 0, np.inf, 0.0))
        worst = max(worst, float(r.max()))
    return worst, float(d.max())


def l1_rel(got, ref, leaf, vol):
    """Per conserved field: sum V |x - x_ref| / sum V |x_ref| over leaf cells."""
    w = (vol * leaf)[:, None]
    num = (w * np.abs(got - ref)).sum(0)
    den = (w * np.abs(ref)).sum(0)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def leaf_and_volume(T):
    leaf = (((T.son_mask[:, None] >> np.arange(8)[None, :]) & 1) == 0).reshape(-1).astype(np.float64)
    vol = np.repeat((0.5 ** T.ijkl[:, 3].astype(np.float64)) ** 3, 8)
    return leaf, vol


def small_trees():
    """(name, ijkl, bc, state-maker) cases small enough for the oracle."""
    gam = 5.0 / 3.0

    def rnd(base, seed):
        def mk(ijkl):
            f = I.random_fields_grid(1 << base, seed, gamma=gam)
            return I.grid_to_tree_state(ijkl, base, f, gam), gam
        return mk

    def sod(ijkl):
        return I.sod_state(ijkl, 1.4), 1.4

    return [
        ("uniform_l4_periodic_random", I.uniform_tree(4), I.PERIODIC, rnd(4, 21)),
        ("uniform_l4_outflow_sod", I.uniform_tree(4), I.OUTFLOW, sod),
        ("amr_3_5_periodic_random", I.sphere_tree(3, 5, (0.4, 0.55, 0.5), 0.22, I.PERIODIC), I.PERIODIC, rnd(3, 22)),
        ("amr_3_5_outflow_random", I.sphere_tree(3, 5, (0.1, 0.2, 0.85), 0.25, I.OUTFLOW), I.OUTFLOW, rnd(3, 23)),
        ("amr_2_5_periodic_wrap", I.sphere_tree(2, 5, (0.02, 0.97, 0.5), 0.2, I.PERIODIC), I.PERIODIC, rnd(2, 24)),
        ("amr_3_5_outflow_sod", I.sphere_tree(3, 5, (0.5, 0.5, 0.5), 0.2, I.OUTFLOW), I.OUTFLOW, sod),
    ]
