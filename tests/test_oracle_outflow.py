"""Pins of the oracle's outflow boundary (reading of the paper, which gives no
hydro boundary condition: zero gradient, an outside position copies the
nearest cell inside the domain).

- Every outside position of every oct's 6^3 tile, on a uniform and on a
  refined outflow tree, against a reference that finds the nearest cell
  inside the domain by its coordinates (at the oct's level, else the coarse
  cell covering it).  A mirror copy (x = -2 taking cell 1) fails it.
- A shock that leaves the box through an outflow wall: the solution inside
  stays the exact Riemann solution of the infinite domain (no reflected
  wave), which a reflecting or periodic wall fails."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I
from refsol import ExactRiemann
from test_oracle_scheme import run_to, to_grid


def _random_cells(n_oct, seed):
    """A state with a different value in every cell (positive density and
    energy), so that copying the wrong cell shows."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(8 * n_oct, 5))
    u[:, 0] = rng.uniform(0.5, 2.0, size=8 * n_oct)
    u[:, 4] = rng.uniform(3.0, 6.0, size=8 * n_oct)
    return u


TREES = [
    ("uniform_l4", lambda: I.uniform_tree(4)),
    ("amr_3_5_corner", lambda: I.sphere_tree(3, 5, (0.1, 0.2, 0.85), 0.25, I.OUTFLOW)),
    ("amr_2_4_face", lambda: I.sphere_tree(2, 4, (0.5, 0.05, 0.5), 0.3, I.OUTFLOW)),
]


@pytest.mark.parametrize("name,mk", TREES, ids=[t[0] for t in TREES])
def test_outside_positions_brute_force(name, mk):
    ijkl = mk()
    T = O.Tree(ijkl, I.OUTFLOW)
    u = _random_cells(T.n, 71)
    cells = {}
    for o in range(T.n):
        i, j, k, l = (int(v) for v in T.ijkl[o])
        for c in range(8):
            cells[(l, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))] = u[8 * o + c]

    def nearest_inside(l, p):
        N = 1 << l
        q = [min(max(v, 0), N - 1) for v in p]
        while (l, *q) not in cells:          # missing oct: the coarse cell under it
            l, q = l - 1, [v >> 1 for v in q]
        return cells[(l, *q)]

    checked = 0
    for o in range(T.n):
        i, j, k, l = (int(v) for v in T.ijkl[o])
        N = 1 << l
        tile = T.tile(u, o)
        for z in range(-2, 4):
            for y in range(-2, 4):
                for x in range(-2, 4):
                    p = [2 * i + x, 2 * j + y, 2 * k + z]
                    if min(p) >= 0 and max(p) < N:
                        continue
                    want = nearest_inside(l, p)
                    assert np.array_equal(tile[z + 2, y + 2, x + 2], want), (name, o, x, y, z)
                    checked += 1
    assert checked > 500


@pytest.mark.parametrize("axis", [0, 2])
def test_shock_leaves_through_outflow_wall(axis):
    """Sod problem with the diaphragm at 0.8 on a 64-cell tube: by t = 0.2
    the shock (speed 1.75) has left through the wall at 1 (at t = 0.114).
    With zero-gradient outflow nothing comes back: the density stays within
    the truncation error of the exact solution of the unbounded problem, and
    the post-shock state between the contact and the wall is the exact one
    (a reflected shock would double the density jump there)."""
    level, x0, t_end = 6, 0.8, 0.2
    ijkl = I.uniform_tree(level)
    T = O.Tree(ijkl, I.OUTFLOW)
    u = T.permute_cells(I.sod_state(ijkl, 1.4, axis=axis, x0=x0))
    with O.threads():
        run_to(T, u, 1.4, 0.8, t_end)
    g = to_grid(T, u)
    # 1-D along the axis: pick the line through the box
    if axis == 0:
        line = g[0, 0, :, :]
    else:
        line = g[:, 0, 0, :]
    N = 1 << level
    x = (np.arange(N) + 0.5) / N
    R = ExactRiemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    rho_ex, u_ex, p_ex = R.sample((x - x0) / t_end)[:3]
    l1 = float(np.mean(np.abs(line[:, 0] - rho_ex)))
    assert l1 < 0.012, l1
    # between the contact (x = 0.8 + 0.9275 t = 0.986) and the rarefaction
    # tail: the star states; the last cells next to the wall hold the
    # post-shock density 0.2656 (exact), far from a reflected shock's ~0.5+
    wall = line[-1, 0]
    assert abs(wall - R.rstar_r) < 0.05, (wall, R.rstar_r)
    # velocity at the wall keeps its sign and size (a reflecting wall sets 0)
    vel = line[-2:, 1 + axis] / line[-2:, 0]
    assert np.all(np.abs(vel - R.ustar) < 0.05), vel
