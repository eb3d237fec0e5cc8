"""Pins of the oracle's multigrid solve on one level of an AMR tree (Sec. 5:
the potential built level by level with V-cycles; the reading of the
boundary data and of the cut cells is stated in the oracle).

- On a complete periodic level it gives the periodic solver's values bit
  for bit (the cut-cell terms vanish and the Dirichlet data is never used).
- Functions that trilinear interpolation reproduces and the 7-point
  Laplacian annihilates (1, x, y, z, xy, yz, zx, xyz) are reproduced
  exactly on a refined patch when the coarse level holds them: a wrong
  interpolation weight, side or index fails this.
- The eigenfunction sin(2 pi x) sin(2 pi y) sin(2 pi z) with f = -12 pi^2 phi
  converges at second order as the patch is refined.
- The fine-level residual equals a brute-force evaluation from the
  definition (neighbour cells found by coordinates in a dictionary, Dirichlet
  data by interpolating the coarse cells found the same way), on a patch
  that wraps across the periodic boundary.
- The masks are the means of +-1 over each cell's descendants, and the
  V-cycle reduces the residual by at least a factor 5 per cycle on refined
  patches (the cut-cell diagonal, the restriction and the prolongation all
  enter this rate)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I


def _centres(T, level):
    idx, cb, ce = O._level_cells(T, level)
    N = 1 << level
    z, y, x = np.unravel_index(idx, (N, N, N))
    return (x + 0.5) / N, (y + 0.5) / N, (z + 0.5) / N, cb, ce


def test_complete_level_equals_periodic_solver():
    L = 4
    T = O.Tree(I.uniform_tree(L), I.PERIODIC)
    rng = np.random.default_rng(1)
    f = rng.standard_normal(8 * T.n)
    f -= f.mean()
    phi = rng.standard_normal(8 * T.n)
    idx, _, _ = O._level_cells(T, L)
    N = 1 << L
    dphi, df = np.zeros(N ** 3), np.zeros(N ** 3)
    dphi[idx], df[idx] = phi, f
    ref, ref_res = O.mg_vcycles(dphi.reshape(N, N, N), df.reshape(N, N, N), 3)
    got = phi.copy()
    res = O.mg_amr_level(T, got, f, L, 3)
    assert np.array_equal(got, ref.reshape(-1)[idx])
    assert np.allclose(res, ref_res, rtol=1e-12)


HARMONIC = {
    "one": lambda x, y, z: 0.75 + 0 * x,
    "x": lambda x, y, z: 1.3 * (x - 0.41),
    "xy": lambda x, y, z: 2.0 * (x - 0.5) * (y - 0.45),
    "yz": lambda x, y, z: -1.5 * (y - 0.52) * (z - 0.55),
    "xyz": lambda x, y, z: 5.0 * (x - 0.5) * (y - 0.48) * (z - 0.5),
    "all": lambda x, y, z: (0.3 + 1.1 * (x - 0.5) - 0.7 * (y - 0.4) + 0.2 * z + 2.0 * (x - 0.5) * (y - 0.45)
                            - 1.5 * (y - 0.5) * (z - 0.55) + 0.8 * (x - 0.4) * (z - 0.6)
                            + 5.0 * (x - 0.5) * (y - 0.5) * (z - 0.5)),
}


@pytest.mark.parametrize("name", list(HARMONIC))
def test_trilinear_harmonics_reproduced(name):
    fn = HARMONIC[name]
    T = O.Tree(I.sphere_tree(4, 5, (0.5, 0.45, 0.55), 0.2, I.PERIODIC), I.PERIODIC)
    phi, f = np.zeros(8 * T.n), np.zeros(8 * T.n)
    x, y, z, cb, ce = _centres(T, 4)
    phi[cb:ce] = fn(x, y, z)
    x, y, z, cb5, ce5 = _centres(T, 5)
    exact = fn(x, y, z)
    O.mg_amr_level(T, phi, f, 5, 30)
    scale = max(np.abs(exact).max(), 1e-3)
    assert np.abs(phi[cb5:ce5] - exact).max() <= 1e-12 * scale


def test_eigenfunction_second_order():
    def ex(x, y, z):
        return np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)

    errs = []
    for base in (3, 4, 5, 6):
        T = O.Tree(I.sphere_tree(base, base + 1, (0.5, 0.45, 0.55), 0.22, I.PERIODIC), I.PERIODIC)
        phi, f = np.zeros(8 * T.n), np.zeros(8 * T.n)
        x, y, z, cb, ce = _centres(T, base)
        phi[cb:ce] = ex(x, y, z)
        x, y, z, cb1, ce1 = _centres(T, base + 1)
        f[cb1:ce1] = -12 * np.pi ** 2 * ex(x, y, z)
        res = O.mg_amr_level(T, phi, f, base + 1, 25)
        assert res[-1] <= 1e-9 * res[0]
        errs.append(np.abs(phi[cb1:ce1] - ex(x, y, z)).max())
    # second order: a factor about 4 per halving of h (the patch's cut
    # differs a little between resolutions)
    assert errs[0] / errs[2] >= 10 and errs[1] / errs[3] >= 10, errs
    assert 2.5 <= errs[2] / errs[3] <= 6.5, errs
    assert errs[3] <= 2e-3, errs


def _brute_residual(T, phi, f, level):
    """f - Lap phi on level `level` from the definition, by coordinates."""
    N, Nc = 1 << level, 1 << (level - 1)
    fine, coarse = {}, {}
    for o in range(T.n):
        i, j, k, l = (int(v) for v in T.ijkl[o])
        for c in range(8):
            p = (2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2))
            if l == level:
                fine[p] = 8 * o + c
            elif l == level - 1:
                coarse[p] = 8 * o + c

    def coarse_phi(I3):
        return phi[coarse[tuple(v % Nc for v in I3)]]

    def value(p):
        p = tuple(v % N for v in p)
        if p in fine:
            return phi[fine[p]]
        C = tuple(v >> 1 for v in p)
        s = tuple(1 if v & 1 else -1 for v in p)
        acc = 0.0
        for b in range(8):
            steps = [(b >> a) & 1 for a in range(3)]
            w = 3 ** (3 - sum(steps)) / 64.0
            acc += w * coarse_phi(tuple(C[a] + steps[a] * s[a] for a in range(3)))
        return acc

    h2 = 0.25 ** level
    out = {}
    for p, cell in fine.items():
        nb = [(p[0] - 1, p[1], p[2]), (p[0] + 1, p[1], p[2]), (p[0], p[1] - 1, p[2]), (p[0], p[1] + 1, p[2]),
              (p[0], p[1], p[2] - 1), (p[0], p[1], p[2] + 1)]
        out[cell] = f[cell] - (sum(value(q) for q in nb) - 6.0 * phi[cell]) / h2
    _, cb, ce = O._level_cells(T, level)
    return np.array([out[c] for c in range(cb, ce)])


@pytest.mark.parametrize("centre", [(0.5, 0.45, 0.55), (0.04, 0.93, 0.5)], ids=["interior", "wrapping"])
def test_fine_residual_brute_force(centre):
    T = O.Tree(I.sphere_tree(3, 4, centre, 0.2, I.PERIODIC), I.PERIODIC)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(8 * T.n)
    f = rng.standard_normal(8 * T.n)
    got = O.mg_amr_residual(T, phi, f, 4)
    ref = _brute_residual(T, phi, f, 4)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_masks_are_descendant_means():
    T = O.Tree(I.sphere_tree(3, 5, (0.3, 0.6, 0.5), 0.2, I.PERIODIC), I.PERIODIC)
    m = O.mg_amr_masks(T, 5, 1)
    idx, _, _ = O._level_cells(T, 5)
    inside = np.zeros(32 ** 3, bool)
    inside[idx] = True
    inside = inside.reshape(32, 32, 32)
    for l in range(1, 5):
        f = 1 << (5 - l)
        counts = inside.reshape(1 << l, f, 1 << l, f, 1 << l, f).sum(axis=(1, 3, 5))
        assert np.array_equal(m[l], (2.0 * counts - f ** 3) / f ** 3), l
    assert np.array_equal(m[5], np.where(inside, 1.0, -1.0))


@pytest.mark.parametrize("shape", [(4, 6, (0.5, 0.45, 0.55), 0.2), (5, 6, (0.1, 0.85, 0.4), 0.18)],
                         ids=["three_levels", "two_levels_wrapping"])
def test_vcycle_rate_level_by_level(shape):
    base, top, centre, radius = shape
    T = O.Tree(I.sphere_tree(base, top, centre, radius, I.PERIODIC), I.PERIODIC)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(8 * T.n)
    cb, ce = 8 * T.level_begin[base], 8 * T.level_begin[base + 1]
    f[cb:ce] -= f[cb:ce].mean()
    phi, res = O.mg_amr_solve(T, f, 6)
    for l, r in res.items():
        rate = (r[-1] / r[1]) ** (1.0 / (len(r) - 2))
        assert rate <= 0.2, (l, r)
    # a level's solve reads only the coarser levels' potential and its own
    # cells: redone alone from the same start it gives the same bits
    again = phi.copy()
    again[8 * T.level_begin[top]:] = 0.0
    O.mg_amr_level(T, again, f, top, 6)
    assert np.array_equal(again, phi)


@pytest.mark.parametrize("m", [3, 4, 5])
def test_coarse_cut_cell_problem_matches_ball_solution(m):
    """The coarse levels' Dirichlet problem, boundary placed by the masks:
    with the fine domain a ball of radius R (cells of level 6 whose centre
    lies inside), Lap e = 1 has the solution (r^2 - R^2) / 6; each coarse
    level reproduces it to within 1% of its largest value (a Neumann-like
    boundary, or one put on the cell faces, does not)."""
    L, R = 6, 0.3
    c = (np.arange(1 << L) + 0.5) / (1 << L)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = ((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) < R * R
    M = 1 << m
    cm = (np.arange(M) + 0.5) / M
    zz, yy, xx = np.meshgrid(cm, cm, cm, indexing="ij")
    exact = (((xx - 0.5) ** 2 + (yy - 0.5) ** 2 + (zz - 0.5) ** 2) - R * R).reshape(-1) / 6.0
    e = O.mg_amr_coarse_sweeps(inside, m, np.ones(M ** 3), np.zeros(M ** 3), 6000)
    ins = O.mg_amr_masks_dense(inside, m) > 0
    assert ins.sum() > 40
    assert np.all(e[~ins] == 0.0)
    assert np.abs(e - exact)[ins].max() <= 1e-2 * np.abs(exact).max()
