"""Pins of the oracle's coarse ghost values (Sec. 2.3 creates ghost zones
where a neighbour oct is missing): injection, and minmod-limited linear
interpolation of the conserved variables inside the coarse cell."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I
from test_oracle_scheme import conserved_uniform, leaf_totals, random_state, run_to

COEF = np.array([[1.0, 0.3, -0.2, 0.1], [0.2, -0.5, 0.4, 0.3], [-0.1, 0.2, 0.6, -0.4], [0.3, 0.1, 0.2, 0.5],
                 [2.5, 0.7, -0.3, 0.2]])     # per variable: a + b x + c y + d z


def _linear(cen):
    return COEF[:, 0] + cen[..., :1] * COEF[:, 1] + cen[..., 1:2] * COEF[:, 2] + cen[..., 2:3] * COEF[:, 3]


def _tile_centres(T, o):
    i, j, k, l = (int(v) for v in T.ijkl[o])
    r = np.arange(-2, 4)
    h = 0.5 ** l
    z, y, x = np.meshgrid((2 * k + r + 0.5) * h, (2 * j + r + 0.5) * h, (2 * i + r + 0.5) * h, indexing="ij")
    return np.stack([x, y, z], -1)


def _coarse_positions(T, o):
    """Tile positions whose value comes from a coarse cell."""
    slot = lambda v: -1 if v < 0 else (1 if v > 1 else 0)
    m = np.zeros((6, 6, 6), bool)
    for z in range(-2, 4):
        for y in range(-2, 4):
            for x in range(-2, 4):
                e = T.nbr27[o][(slot(x) + 1) + 3 * (slot(y) + 1) + 9 * (slot(z) + 1)]
                m[z + 2, y + 2, x + 2] = e < 0 and e != O.OUTSIDE
    return m


def _two_level():
    ijkl = I.sphere_tree(3, 4, (0.5, 0.5, 0.5), 0.22, I.OUTFLOW)
    cen, _ = I.cell_centres(ijkl)
    u = I.fill_split_cells(ijkl, _linear(cen).reshape(-1, 5))
    return ijkl, u


def test_linear_field_is_reproduced():
    """A field linear in space: inside the domain every tile value, coarse
    ghosts included, is the field at the fine position (interpolation is
    exact for linear data); injection misses the coarse positions by a
    quarter of the coarse difference."""
    ijkl, u_in = _two_level()
    checked = 0
    for mode in (O.GHOST_LINEAR, O.GHOST_INJECT):
        T = O.Tree(ijkl, I.OUTFLOW, ghost=mode)
        u = T.permute_cells(u_in)
        for o in range(T.n):
            if T.ijkl[o, 3] != T.lmax:
                continue
            cen = _tile_centres(T, o)
            if cen.min() < 0 or cen.max() > 1:
                continue
            coarse = _coarse_positions(T, o)
            if not coarse.any():
                continue
            want = _linear(cen)
            got = T.tile(u, o)
            err = np.abs(got - want).max(-1)
            if mode == O.GHOST_LINEAR:
                assert err.max() <= 1e-14, (o, err.max())
                checked += 1
            else:
                assert err[~coarse].max() <= 1e-14
                assert err[coarse].min() > 1e-3
    assert checked > 10


def test_extremum_gives_injection():
    """At a coarse cell that is a local maximum along every axis, minmod
    gives zero slopes and every fine position takes the cell's values."""
    ijkl, _ = _two_level()
    T = O.Tree(ijkl, I.OUTFLOW, ghost=O.GHOST_LINEAR)
    u = conserved_uniform(8 * T.n, 1.0, (0.0, 0.0, 0.0), 1.0, 1.4)
    o = next(q for q in range(T.n) if T.ijkl[q, 3] == T.lmax and _coarse_positions(T, q).any()
             and _tile_centres(T, q).min() > 0 and _tile_centres(T, q).max() < 1)
    coarse = _coarse_positions(T, o)
    z, y, x = np.argwhere(coarse)[0] - 2
    slot = lambda v: -1 if v < 0 else (1 if v > 1 else 0)
    C = -1 - T.nbr27[o][(slot(x) + 1) + 3 * (slot(y) + 1) + 9 * (slot(z) + 1)]
    u[C] *= 2.0
    tile = T.tile(u, o)
    src = np.zeros((6, 6, 6), bool)
    for zz in range(-2, 4):
        for yy in range(-2, 4):
            for xx in range(-2, 4):
                src[zz + 2, yy + 2, xx + 2] = coarse[zz + 2, yy + 2, xx + 2] and \
                    -1 - T.nbr27[o][(slot(xx) + 1) + 3 * (slot(yy) + 1) + 9 * (slot(zz) + 1)] == C
    assert src.sum() >= 1
    assert np.all(tile[src] == u[C])


AMR = [
    ("amr_3_5_periodic", lambda: I.sphere_tree(3, 5, (0.4, 0.55, 0.5), 0.2, I.PERIODIC), I.PERIODIC),
    ("amr_3_5_outflow", lambda: I.sphere_tree(3, 5, (0.1, 0.2, 0.85), 0.25, I.OUTFLOW), I.OUTFLOW),
]


@pytest.mark.parametrize("name,mk,bc", AMR, ids=[t[0] for t in AMR])
def test_uniform_states(name, mk, bc):
    T = O.Tree(mk(), bc, ghost=O.GHOST_LINEAR)
    u = conserved_uniform(8 * T.n, 1.3, (0.0, 0.0, 0.0), 0.7, 1.4)
    u0 = u.copy()
    T.run(u, 1.4, 0.8, 3)
    assert np.array_equal(u, u0)
    u = conserved_uniform(8 * T.n, 0.9, (0.7, -0.4, 0.25), 1.1, 5.0 / 3.0)
    u0 = u.copy()
    T.run(u, 5.0 / 3.0, 0.8, 3)
    assert np.all(np.abs(u - u0) <= 8 * np.finfo(float).eps * np.abs(u0).max(0))


@pytest.mark.parametrize("subcycled", [False, True])
def test_conservation(subcycled):
    ijkl = I.sphere_tree(3, 5, (0.45, 0.5, 0.6), 0.22, I.PERIODIC)
    T = O.Tree(ijkl, I.PERIODIC, ghost=O.GHOST_LINEAR)
    gam = 5.0 / 3.0
    u = T.permute_cells(random_state(ijkl, 3, 11, gam))
    tot0, abs0 = leaf_totals(T, u)
    for _ in range(3):
        (T.step_subcycled if subcycled else T.step)(u, gam, 0.8)
    tot, absv = leaf_totals(T, u)
    assert np.all(np.abs(tot - tot0) <= 1e-13 * np.maximum(abs0, absv))


def test_interpolation_lowers_the_crossing_error():
    """A density pulse advected through a refined sphere: with interpolated
    coarse ghosts the refined region tracks the exact profile better than
    with injected ones (measured: 10 % lower L1 error there)."""
    gam = 1.4
    ijkl = I.sphere_tree(4, 5, (0.55, 0.5, 0.5), 0.2, I.PERIODIC)

    def err(mode):
        T = O.Tree(ijkl, I.PERIODIC, ghost=mode)
        cen, _ = I.cell_centres(ijkl)
        x = cen[..., 0]
        rho = 1.0 + 0.5 * np.exp(-((x - 0.3) ** 2) / (2 * 0.06 ** 2))
        z = np.zeros_like(rho)
        u = T.permute_cells(I.fill_split_cells(ijkl, I.conserved(rho, z + 1.0, z, z, z + 1.0, gam).reshape(-1, 5)))
        run_to(T, u, gam, 0.8, 0.4)
        cen, _ = I.cell_centres(T.ijkl)
        exact = 1.0 + 0.5 * np.exp(-((cen[..., 0].reshape(-1) - 0.7) ** 2) / (2 * 0.06 ** 2))
        leaf = (((T.son_mask[:, None] >> np.arange(8)[None, :]) & 1) == 0).reshape(-1)
        fine = np.repeat(T.ijkl[:, 3] == T.lmax, 8)
        vol = np.repeat((0.5 ** T.ijkl[:, 3].astype(float)) ** 3, 8)
        return float(np.sum((vol * np.abs(u[:, 0] - exact))[leaf & fine]))

    # L1 error over the refined region, whose inflow passes the coarse ghosts
    e_inj, e_lin = err(O.GHOST_INJECT), err(O.GHOST_LINEAR)
    assert e_lin < 0.95 * e_inj, (e_lin, e_inj)


def test_sedov_symmetry_linear():
    w = I.sedov_amr(base=4, lmax=6, radius=0.15)
    T = O.Tree(w.ijkl, w.bc, ghost=O.GHOST_LINEAR)
    u = T.permute_cells(w.u)
    T.run(u, w.gamma, w.cfl, 10)
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


def _minmod(a, b):
    same = ((a > 0) & (b > 0)) | ((a < 0) & (b < 0))
    return np.where(same, np.copysign(np.minimum(np.abs(a), np.abs(b)), a), 0.0)


@pytest.mark.parametrize("bc", [I.PERIODIC, I.OUTFLOW])
@pytest.mark.parametrize("mode", [O.GHOST_INJECT, O.GHOST_LINEAR])
def test_coarse_ghosts_brute_force(bc, mode):
    """Every coarse-ghost position of every oct of a three-level tree with a
    random state, against a reference that finds cells by their coordinates
    (the coarse cell under the position, its face neighbours at its level or
    the coarser cell covering them, itself across an outflow face) and
    applies the definition with numpy."""
    centre = (0.45, 0.5, 0.55) if bc == I.PERIODIC else (0.12, 0.2, 0.8)
    ijkl = I.sphere_tree(3, 5, centre, 0.22, bc)
    T = O.Tree(ijkl, bc, ghost=mode)
    u = T.permute_cells(random_state(ijkl, 3, 61, 5.0 / 3.0))
    cells = {}
    for o in range(T.n):
        i, j, k, l = (int(v) for v in T.ijkl[o])
        for c in range(8):
            cells[(l, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))] = u[8 * o + c]

    def at(l, p):
        N = 1 << l
        if bc == I.PERIODIC:
            p = [q % N for q in p]
        elif min(p) < 0 or max(p) >= N:
            return None
        while (l, *p) not in cells:
            l, p = l - 1, [q >> 1 for q in p]
        return cells[(l, *p)]

    checked = 0
    for o in range(T.n):
        coarse = _coarse_positions(T, o)
        if not coarse.any():
            continue
        i, j, k, l = (int(v) for v in T.ijkl[o])
        tile = T.tile(u, o)
        N = 1 << l
        for z, y, x in np.argwhere(coarse):
            p = [2 * i + x - 2, 2 * j + y - 2, 2 * k + z - 2]
            if bc == I.PERIODIC:
                p = [q % N for q in p]
            else:
                p = [min(max(q, 0), N - 1) for q in p]
            assert (l, *p) not in cells
            cp = [q >> 1 for q in p]
            uc = cells[(l - 1, *cp)]
            want = uc.copy()
            if mode == O.GHOST_LINEAR:
                for a in range(3):
                    lo, hi = list(cp), list(cp)
                    lo[a] -= 1
                    hi[a] += 1
                    ul, ur = at(l - 1, lo), at(l - 1, hi)
                    ul = uc if ul is None else ul
                    ur = uc if ur is None else ur
                    want = want + (0.25 if p[a] & 1 else -0.25) * _minmod(uc - ul, ur - uc)
            assert np.array_equal(tile[z, y, x], want), (o, x, y, z)
            checked += 1
    assert checked > 100
