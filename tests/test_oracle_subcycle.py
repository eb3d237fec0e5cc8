"""Pins of the oracle's subcycled step (Sec. 2: adaptive time steps level by
level, each level two steps of half its parent's): exact reductions to the
global step, exact invariants, and the step size against brute force."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I
from test_oracle_scheme import conserved_uniform, leaf_totals, random_state


def _eq_or_report(a, b):
    d = np.nonzero(np.any(a != b, axis=1))[0]
    assert d.size == 0, "%d cells differ, first %s" % (d.size, d[:8])


@pytest.mark.parametrize("bc", [I.PERIODIC, I.OUTFLOW])
def test_single_level_equals_global_step(bc):
    """With one level there is nothing to subcycle: the step and its dt are
    the global step's, bit for bit."""
    ijkl = I.uniform_tree(4)
    T = O.Tree(ijkl, bc)
    gam = 5.0 / 3.0
    u = T.permute_cells(random_state(ijkl, 4, 21, gam))
    v = u.copy()
    for _ in range(3):
        assert T.cfl_dt_subcycled(u, gam, 0.8) == T.cfl_dt(u, gam, 0.8)
        d1 = T.step_subcycled(u, gam, 0.8)
        d2 = T.step(v, gam, 0.8)
        assert d1 == d2
        _eq_or_report(u, v)


AMR = [
    ("amr_3_5_periodic", lambda: I.sphere_tree(3, 5, (0.4, 0.55, 0.5), 0.2, I.PERIODIC), I.PERIODIC),
    ("amr_3_5_outflow", lambda: I.sphere_tree(3, 5, (0.1, 0.2, 0.85), 0.25, I.OUTFLOW), I.OUTFLOW),
    ("amr_3_6_periodic", lambda: I.sphere_tree(3, 6, (0.5, 0.45, 0.5), 0.15, I.PERIODIC), I.PERIODIC),
]


@pytest.mark.parametrize("name,mk,bc", AMR, ids=[t[0] for t in AMR])
def test_uniform_state_at_rest_is_exact(name, mk, bc):
    T = O.Tree(mk(), bc)
    u = conserved_uniform(8 * T.n, 1.3, (0.0, 0.0, 0.0), 0.7, 1.4)
    u0 = u.copy()
    T.run_subcycled(u, 1.4, 0.8, 3)
    _eq_or_report(u, u0)


@pytest.mark.parametrize("name,mk,bc", AMR, ids=[t[0] for t in AMR])
def test_uniform_moving_state(name, mk, bc):
    """A coarse cell on a coarse-fine face gets its flux there from the two
    fine substeps; a uniform flow is kept to a few ulp."""
    T = O.Tree(mk(), bc)
    u = conserved_uniform(8 * T.n, 0.9, (0.7, -0.4, 0.25), 1.1, 5.0 / 3.0)
    u0 = u.copy()
    T.run_subcycled(u, 5.0 / 3.0, 0.8, 3)
    assert np.all(np.abs(u - u0) <= 8 * np.finfo(float).eps * np.abs(u0).max(0))


@pytest.mark.parametrize("lmax", [5, 6])
def test_conservation(lmax):
    """Leaf sums of volume * (mass, momentum, energy) stay constant to
    rounding with two or three refined levels and Mach-2 random flow: the
    fine fluxes of both substeps reach the coarse side.  Dropping either
    substep's share, or scaling it, breaks this at order one.  The global
    step drifts by the same few 1e-14 on these trees."""
    ijkl = I.sphere_tree(3, lmax, (0.45, 0.5, 0.6), 0.22, I.PERIODIC)
    T = O.Tree(ijkl, I.PERIODIC)
    assert T.lmax == lmax
    gam = 5.0 / 3.0
    u = T.permute_cells(random_state(ijkl, 3, 11, gam))
    tot0, abs0 = leaf_totals(T, u)
    for _ in range(4):
        T.step_subcycled(u, gam, 0.8)
        tot, absv = leaf_totals(T, u)
        assert np.all(np.abs(tot - tot0) <= 1e-13 * np.maximum(abs0, absv))


def test_dt_brute_force():
    """The coarse step is the smallest leaf limit CFL dx_l / (|u|+|v|+|w|+3c)
    scaled by 2^(l - lmin), the factor by which level l's own step is
    smaller."""
    gam = 1.4
    ijkl = I.sphere_tree(3, 5, (0.5, 0.5, 0.5), 0.2, I.PERIODIC)
    T = O.Tree(ijkl, I.PERIODIC)
    u = T.permute_cells(random_state(ijkl, 3, 5, gam))
    rho = np.maximum(u[:, 0], 1e-10)
    vel = u[:, 1:4] / rho[:, None]
    p = np.maximum((gam - 1) * (u[:, 4] - 0.5 * rho * (vel ** 2).sum(1)), 1e-20)
    lev = np.repeat(T.ijkl[:, 3].astype(float), 8)
    dx = 0.5 ** lev
    leaf = (((T.son_mask[:, None] >> np.arange(8)[None, :]) & 1) == 0).reshape(-1)
    cand = dx / (np.abs(vel).sum(1) + 3 * np.sqrt(gam * p / rho)) * 2.0 ** (lev - T.lmin)
    want = 0.8 * cand[leaf].min()
    got = T.cfl_dt_subcycled(u, gam, 0.8)
    assert abs(got - want) <= 4 * np.finfo(float).eps * want
    # never smaller than the global step, at most 2^(lmax - lmin) times it
    g = T.cfl_dt(u, gam, 0.8)
    assert g * (1 - 1e-15) <= got <= g * 2 ** (T.lmax - T.lmin) * (1 + 1e-15)


@pytest.mark.parametrize("lmax", [4, 5])
def test_fine_blast_equals_small_global_steps(lmax):
    """A pressure spike on a few finest cells, deep inside the finest region,
    in gas at rest.  For one coarse step nothing reaches a coarser cell, so
    the coarser levels stay exactly at rest and the finest level sees the
    same ghosts either way: one subcycled step of size D must equal
    2^(lmax - lmin) global steps of size D / 2^(lmax - lmin), bit for bit.
    Tests the per-level step size, the number of substeps and the order of
    the recursion."""
    gam = 1.4
    ijkl = I.sphere_tree(3, lmax, (0.5, 0.5, 0.5), 0.45, I.PERIODIC)
    T = O.Tree(ijkl, I.PERIODIC)
    assert (T.lmin, T.lmax) == (3, lmax)
    cen, h = I.cell_centres(T.ijkl)
    fine = T.ijkl[:, 3] == lmax
    hf = 0.5 ** lmax
    spike = np.all(np.abs(cen - 0.5) < 1.6 * hf, axis=-1) & fine[:, None]
    assert spike.sum() == 64
    z = np.zeros(cen.shape[:2])
    u = I.conserved(1.0 + z, z, z, z, np.where(spike, 10.0, 1.0), gam).reshape(-1, 5)
    u = np.ascontiguousarray(I.fill_split_cells(T.ijkl, u))
    u0 = u.copy()
    v = u.copy()
    D = T.cfl_dt_subcycled(u, gam, 0.8)
    k = 2 ** (lmax - T.lmin)
    assert D == k * T.cfl_dt(u, gam, 0.8)
    assert T.step_subcycled(u, gam, 0.8) == D
    for _ in range(k):
        T.step_fixed(v, gam, D / k)
    _eq_or_report(u, v)
    # the spike moved, and no coarser leaf cell changed (split cells hold
    # the restriction of the finest level)
    changed = np.any(u != u0, axis=1).reshape(-1, 8)
    leaf = ((T.son_mask[:, None] >> np.arange(8)[None, :]) & 1) == 0
    assert changed[fine].sum() > 64
    assert not (changed & leaf)[~fine].any()
    assert (changed & ~leaf).any()


def test_sedov_symmetry():
    """The Sedov tree and state are symmetric about the three mid-planes and
    stay so (to rounding) through subcycled steps."""
    w = I.sedov_amr(base=4, lmax=6, radius=0.15)
    T = O.Tree(w.ijkl, w.bc)
    u = T.permute_cells(w.u)
    T.run_subcycled(u, w.gamma, w.cfl, 6)
    pos = {}
    for o in range(T.n):
        i, j, k, l = T.ijkl[o]
        for c in range(8):
            pos[(l, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))] = 8 * o + c
    scale = np.abs(u).max(0) + 1e-300
    worst = 0.0
    for (l, x, y, z), cell in pos.items():
        N = (1 << l) - 1
        for axis in range(3):
            m = [x, y, z]
            m[axis] = N - m[axis]
            b = u[pos[(l, *m)]].copy()
            b[1 + axis] *= -1
            worst = max(worst, float(np.max(np.abs(u[cell] - b) / scale)))
    assert worst <= 1e-13
