"""Seeded synthetic workloads: oct trees and initial conserved states.

This module holds only input generation (tree geometry and initial conditions),
none of the hydro method's arithmetic; both the HIP path and the CPU oracle
consume its output byte for byte.

A tree is an int32 array ``ijkl[n, 4]`` of octs (i, j, k, level) in *input
order*: by level, then lexicographic in (k, j, i).  Level l has 2^l cells and
2^(l-1) octs per side of the unit box.  The state is ``u[8n, 5]`` float64 with
cell id 8*oct + ix + 2*iy + 4*iz and variables (rho, rho u, rho v, rho w, E).

Trees are graded: every cell that has children has all 26 same-level
neighbours present (after periodic wrap, or clipped at outflow walls), so every
missing neighbour of an oct is covered by a coarse leaf cell.  Split cells hold
the mean of their children.
"""
import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, OUTFLOW = 0, 1


# --------------------------------------------------------------------------
# tree geometry
# --------------------------------------------------------------------------

def _code(i, j, k, N):
    return (np.asarray(k, np.int64) * N + np.asarray(j, np.int64)) * N + np.asarray(i, np.int64)


def _decode(c, N):
    c = np.asarray(c, np.int64)
    return c % N, (c // N) % N, c // (N * N)


def _cell_centres(level, octs_ijk):
    """Centres (x, y, z) of the 8 cells of each oct, shape [n, 8, 3]."""
    h = 1.0 / (1 << level)
    o = np.asarray(octs_ijk, np.float64).reshape(-1, 1, 3)
    sub = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.float64).reshape(1, 8, 3)
    return (2.0 * o + sub + 0.5) * h


def _close(levels, lmin, bc):
    """Grading closure, finest level first: the father cell of every oct at
    level l+1 needs its 26 neighbours at level l, whose octs are added."""
    lmax = max(levels)
    for l in range(lmax - 1, lmin, -1):
        fine = levels.get(l + 1)
        if fine is None or len(fine) == 0:
            continue
        Nf = 1 << l              # octs per side at level l+1 == cells per side at level l
        fi, fj, fk = _decode(fine, Nf)
        need = [levels.get(l, np.zeros(0, np.int64))]
        No = 1 << (l - 1)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ci, cj, ck = fi + dx, fj + dy, fk + dz
                    if bc == PERIODIC:
                        ci, cj, ck = ci % Nf, cj % Nf, ck % Nf
                        keep = np.ones(len(ci), bool)
                    else:
                        keep = (ci >= 0) & (ci < Nf) & (cj >= 0) & (cj < Nf) & (ck >= 0) & (ck < Nf)
                    need.append(_code(ci[keep] >> 1, cj[keep] >> 1, ck[keep] >> 1, No))
        levels[l] = np.unique(np.concatenate(need))
    return levels


def _levels_to_ijkl(levels):
    parts = []
    for l in sorted(levels):
        codes = np.sort(levels[l])
        i, j, k = _decode(codes, 1 << (l - 1))
        parts.append(np.stack([i, j, k, np.full(len(codes), l)], axis=1))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.int32))


def uniform_tree(level):
    """All octs of one level (2^(3(level-1)) octs)."""
    N = 1 << (level - 1)
    return _levels_to_ijkl({level: np.arange(N ** 3, dtype=np.int64)})


def full_tree(level):
    """Every oct of levels 1..level (each cell below `level` split): the
    hierarchy of a multigrid solver on a level-`level` unigrid."""
    return _levels_to_ijkl({l: np.arange(8 ** (l - 1), dtype=np.int64) for l in range(1, level + 1)})


def _siblings(levels, base):
    """Every oct above `base` brings its 7 siblings (4^3-cell blocks)."""
    for l in sorted(levels):
        if l <= base or len(levels[l]) == 0:
            continue
        i, j, k = _decode(levels[l], 1 << (l - 1))
        kids = [_code(2 * (i >> 1) + a, 2 * (j >> 1) + b, 2 * (k >> 1) + c, 1 << (l - 1))
                for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        levels[l] = np.unique(np.concatenate([levels[l]] + kids))
    return levels


def refined_tree(base, lmax, flag, bc, max_passes=8, blocks=False):
    """Base level complete; a cell of level l < lmax is refined when
    ``flag(l, centres[m,3]) -> bool[m]`` says so and its oct exists; graded
    closure is applied and flagging repeated until nothing changes.  With
    blocks=True an oct's cells are refined together (a flag on one flags all
    eight) and every oct comes with its siblings."""
    levels = {base: np.arange((1 << (base - 1)) ** 3, dtype=np.int64)}
    for _ in range(max_passes if not blocks else 4 * max_passes):
        before = {l: len(v) for l, v in levels.items()}
        for l in range(base, lmax):
            octs = levels.get(l)
            if octs is None or len(octs) == 0:
                break
            i, j, k = _decode(octs, 1 << (l - 1))
            cen = _cell_centres(l, np.stack([i, j, k], 1))
            f = flag(l, cen.reshape(-1, 3)).reshape(-1, 8)
            if blocks:
                f = np.repeat(f.any(1, keepdims=True), 8, axis=1)
            oo, cc = np.nonzero(f)
            ci = 2 * i[oo] + (cc & 1)
            cj = 2 * j[oo] + ((cc >> 1) & 1)
            ck = 2 * k[oo] + ((cc >> 2) & 1)
            new = _code(ci, cj, ck, 1 << l)
            levels[l + 1] = np.unique(np.concatenate([levels.get(l + 1, np.zeros(0, np.int64)), new]))
        levels = _close(levels, base, bc)
        if blocks:
            levels = _siblings(levels, base)
        if {l: len(v) for l, v in levels.items()} == before:
            break
    return _levels_to_ijkl({l: v for l, v in levels.items() if len(v)})


def sphere_tree(base, lmax, centre, radius, bc, blocks=False):
    """Refine every cell whose centre lies within `radius` of `centre`
    (minimum-image distance for periodic boxes) up to level lmax."""
    c = np.asarray(centre, np.float64).reshape(1, 3)

    def flag(l, cen):
        d = cen - c
        if bc == PERIODIC:
            d = d - np.round(d)
        return (d * d).sum(1) < radius * radius

    return refined_tree(base, lmax, flag, bc, blocks=blocks)


def split_info(ijkl):
    """For each oct above the coarsest level: (father oct index, cell bit) in
    input order, found by coordinate lookup."""
    ijkl = np.asarray(ijkl)
    lv = ijkl[:, 3]
    fo = np.full(len(ijkl), -1, np.int64)
    fb = np.zeros(len(ijkl), np.int64)
    for l in np.unique(lv):
        if l == lv.min():
            continue
        sel = np.nonzero(lv == l)[0]
        par = np.nonzero(lv == l - 1)[0]
        Np = 1 << (l - 2)
        pc = _code(ijkl[par, 0], ijkl[par, 1], ijkl[par, 2], Np)
        order = np.argsort(pc)
        q = _code(ijkl[sel, 0] >> 1, ijkl[sel, 1] >> 1, ijkl[sel, 2] >> 1, Np)
        pos = np.searchsorted(pc[order], q)
        if np.any(pos >= len(par)) or np.any(pc[order][np.minimum(pos, len(par) - 1)] != q):
            raise ValueError("oct without father at level %d" % l)
        fo[sel] = par[order[pos]]
        fb[sel] = (ijkl[sel, 0] & 1) + 2 * (ijkl[sel, 1] & 1) + 4 * (ijkl[sel, 2] & 1)
    return fo, fb


def fill_split_cells(ijkl, u):
    """Give every split cell the mean of its child oct's 8 cells, finest
    level first (initial data only)."""
    u = u.reshape(-1, 8, 5)
    fo, fb = split_info(ijkl)
    lv = np.asarray(ijkl)[:, 3]
    for l in sorted(np.unique(lv))[::-1]:
        sel = np.nonzero((lv == l) & (fo >= 0))[0]
        if len(sel):
            u[fo[sel], fb[sel], :] = u[sel].mean(axis=1)
    return u.reshape(-1, 5)


def cell_centres(ijkl):
    """[n, 8, 3] centres and [n] cell widths of every cell, input order."""
    ijkl = np.asarray(ijkl)
    cen = np.empty((len(ijkl), 8, 3))
    for l in np.unique(ijkl[:, 3]):
        sel = ijkl[:, 3] == l
        cen[sel] = _cell_centres(int(l), ijkl[sel, :3])
    return cen, 1.0 / (1 << ijkl[:, 3]).astype(np.float64)


def leaf_mask(ijkl):
    """[n, 8] bool, True where the cell has no child oct."""
    fo, fb = split_info(ijkl)
    m = np.ones((len(ijkl), 8), bool)
    sel = fo >= 0
    m[fo[sel], fb[sel]] = False
    return m


# --------------------------------------------------------------------------
# initial states
# --------------------------------------------------------------------------

def conserved(rho, vx, vy, vz, p, gamma):
    e = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, e], axis=-1)


def sod_state(ijkl, gamma=1.4, axis=0, x0=0.5):
    """Sod tube along `axis`: (rho, p) = (1, 1) where the cell centre is below
    x0, (0.125, 0.1) above; at rest."""
    cen, _ = cell_centres(ijkl)
    left = cen[..., axis] < x0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros_like(rho)
    u = conserved(rho, z, z, z, p, gamma).reshape(-1, 5)
    return fill_split_cells(ijkl, u)


def sedov_state(ijkl, gamma=1.4, energy=1.0, p0=1e-5, rho0=1.0):
    """Uniform gas at rest; `energy` deposited as thermal energy, shared
    equally by the 8 finest cells that touch the box centre."""
    ijkl = np.asarray(ijkl)
    cen, h = cell_centres(ijkl)
    z = np.zeros(cen.shape[:2])
    u = conserved(rho0 + z, z, z, z, p0 + z, gamma)
    lmax = ijkl[:, 3].max()
    fine = ijkl[:, 3] == lmax
    hmax = 1.0 / (1 << lmax)
    near = np.all(np.abs(cen - 0.5) < 0.75 * hmax, axis=-1) & fine[:, None]
    if near.sum() != 8:
        raise ValueError("expected 8 finest cells around the centre, found %d" % near.sum())
    u[near, 4] = energy / 8.0 / hmax ** 3
    return fill_split_cells(ijkl, u.reshape(-1, 5))


def _filtered_noise(rng, N, slope):
    """White noise on an N^3 grid filtered to |f(k)|^2 ~ k^slope for
    1 <= |k| <= N/2, zero mean, unit variance."""
    noise = rng.standard_normal((N, N, N))
    f = np.fft.rfftn(noise)
    k1 = np.fft.fftfreq(N) * N
    k3 = np.fft.rfftfreq(N) * N
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k3[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    band = (kk >= 1.0) & (kk <= N / 2)
    amp[band] = kk[band] ** (slope / 2.0)
    f *= amp
    g = np.fft.irfftn(f, s=(N, N, N), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def random_fields_grid(N, seed, sigma_ln=0.5, mach=2.0, p=1.0, gamma=5.0 / 3.0, slope=-4.0):
    """Lognormal density (ln rho = sigma g - sigma^2/2) and Gaussian
    random-phase velocities with E(k) ~ k^-2 (|v(k)|^2 ~ k^-4), rms |v| =
    mach * sqrt(gamma p / mean rho); uniform pressure.  Arrays indexed [z, y, x]."""
    rng = np.random.default_rng(seed)
    g = _filtered_noise(rng, N, slope)
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln ** 2)
    vel = [_filtered_noise(rng, N, slope) for _ in range(3)]
    rms = np.sqrt(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    scale = mach * np.sqrt(gamma * p / 1.0) / rms
    vel = [v * scale for v in vel]
    return rho, vel[0], vel[1], vel[2], np.full_like(rho, p)


def grid_to_tree_state(ijkl, grid_level, fields, gamma):
    """Sample per-cell fields given on the uniform grid of `grid_level`
    ([z, y, x] arrays) onto the leaf cells of the tree: a cell at the grid
    level takes its own value, a finer cell takes the value of the grid cell
    that contains it (injection); split cells are then set to the mean of
    their children."""
    ijkl = np.asarray(ijkl)
    cen, _ = cell_centres(ijkl)
    N = 1 << grid_level
    idx = np.minimum((cen * N).astype(np.int64), N - 1)
    vals = [f[idx[..., 2], idx[..., 1], idx[..., 0]] for f in fields]
    u = conserved(*vals, gamma).reshape(-1, 5)
    return fill_split_cells(ijkl, u)


class ClumpField:
    """Uniform background plus Gaussian clumps:
    rho(x) = 1 + sum_c A_c prod_axes exp(-d_a^2 / (2 R_c^2)),
    d_a the minimum-image distance to clump centre c along axis a (periodic
    unit box).  Centres uniform, radii R uniform in [r_min, r_max] cells of
    `base_level`, amplitudes lognormal A = exp(sigma_a g)."""

    def __init__(self, nclump, seed, sigma_a, base_level, r_cells=(2.0, 20.0)):
        rng = np.random.default_rng(seed)
        self.centre = rng.uniform(0.0, 1.0, (nclump, 3))
        self.radius = rng.uniform(r_cells[0], r_cells[1], nclump) / (1 << base_level)
        self.amp = np.exp(sigma_a * rng.standard_normal(nclump))

    def mean(self):
        """Box average of rho (each clump integrates to A (sqrt(2 pi) R
        erf(1 / (2 sqrt 2 R)))^3 over its minimum-image cell)."""
        one = np.array([math.sqrt(2.0 * math.pi) * r * math.erf(1.0 / (2.0 * math.sqrt(2.0) * r))
                        for r in self.radius])
        return 1.0 + float(np.sum(self.amp * one ** 3))

    def _axis(self, level, axis):
        n = 1 << level
        x = (np.arange(n) + 0.5) / n
        d = x[None, :] - self.centre[:, axis:axis + 1]
        d -= np.round(d)
        return np.exp(-0.5 * (d / self.radius[:, None]) ** 2)

    def at_cells(self, level, ci, cj, ck, tile=16, batch=16):
        """rho at the centres of the level-`level` cells (ci, cj, ck): the
        separable sum is evaluated on the tile x tile x tile blocks that hold
        the requested cells, as one matrix product per block."""
        ci, cj, ck = (np.asarray(a, np.int64) for a in (ci, cj, ck))
        if len(ci) == 0:
            return np.zeros(0)
        n = 1 << level
        t = min(tile, n)
        nt = n // t
        ex, ey, ez = (self._axis(level, a) for a in range(3))
        tid = ((ck // t) * nt + (cj // t)) * nt + (ci // t)
        tiles, inv = np.unique(tid, return_inverse=True)
        tx, ty, tz = tiles % nt, (tiles // nt) % nt, tiles // (nt * nt)
        ar = np.arange(t)
        vals = np.empty((len(tiles), t, t, t))
        for b0 in range(0, len(tiles), batch):
            sl = slice(b0, min(b0 + batch, len(tiles)))
            I, J, K = tx[sl, None] * t + ar, ty[sl, None] * t + ar, tz[sl, None] * t + ar
            X = ex[:, I].transpose(1, 2, 0)                                      # [b, i, c]
            Y = ey[:, J].transpose(1, 0, 2)[:, :, :, None]                       # [b, c, j, 1]
            Z = ez[:, K].transpose(1, 0, 2)[:, :, None, :]                       # [b, c, 1, k]
            M = (self.amp[None, :, None, None] * Y * Z).reshape(len(I), len(self.amp), t * t)
            vals[sl] = (X @ M).reshape(len(I), t, t, t)                          # [b, i, j, k]
        return 1.0 + vals[inv, ci % t, cj % t, ck % t]


def _oct_cells(octs, level):
    """Cell indices (ci, cj, ck) of the 8 cells of each oct code, [n*8]."""
    i, j, k = _decode(octs, 1 << (level - 1))
    c = np.arange(8)
    return ((2 * i[:, None] + (c & 1)).ravel(), (2 * j[:, None] + ((c >> 1) & 1)).ravel(),
            (2 * k[:, None] + ((c >> 2) & 1)).ravel())


def clump_tree(fieldobj, base, lmax, threshold, max_passes=8):
    """Periodic tree refined cell by cell wherever rho(cell centre) >
    `threshold`, from the complete `base` level up to `lmax`, with the grading
    closure; flagging is repeated for octs the closure adds.  Returns (ijkl,
    {level: (oct codes, rho of their 8 cells)})."""
    levels = {base: np.arange((1 << (base - 1)) ** 3, dtype=np.int64)}
    rho = {}          # level -> dict code -> row in a values array
    cache = {}

    def values(l, octs):
        codes, vals = cache.get(l, (np.zeros(0, np.int64), np.zeros((0, 8))))
        new = np.setdiff1d(octs, codes, assume_unique=True)
        if len(new):
            v = fieldobj.at_cells(l, *_oct_cells(new, l)).reshape(-1, 8)
            codes = np.concatenate([codes, new])
            vals = np.concatenate([vals, v])
            order = np.argsort(codes)
            codes, vals = codes[order], vals[order]
            cache[l] = (codes, vals)
        pos = np.searchsorted(codes, octs)
        return vals[pos]

    for _ in range(max_passes):
        before = {l: len(v) for l, v in levels.items()}
        for l in range(base, lmax):
            octs = levels.get(l)
            if octs is None or len(octs) == 0:
                break
            f = values(l, octs) > threshold
            oo, cc = np.nonzero(f)
            i, j, k = _decode(octs[oo], 1 << (l - 1))
            new = _code(2 * i + (cc & 1), 2 * j + ((cc >> 1) & 1), 2 * k + ((cc >> 2) & 1), 1 << l)
            levels[l + 1] = np.unique(np.concatenate([levels.get(l + 1, np.zeros(0, np.int64)), new]))
        levels = _close(levels, base, PERIODIC)
        if {l: len(v) for l, v in levels.items()} == before:
            break
    levels = {l: v for l, v in levels.items() if len(v)}
    for l, octs in levels.items():
        rho[l] = (np.sort(octs), values(l, np.sort(octs)))
    return _levels_to_ijkl(levels), rho


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ijkl: np.ndarray          # [n, 4] int32, input order
    u: np.ndarray             # [8n, 5] float64, input order
    gamma: float
    cfl: float
    bc: int
    nsteps: int
    meta: dict = field(default_factory=dict)

    @property
    def n_oct(self):
        return len(self.ijkl)

    @property
    def n_cell(self):
        return 8 * len(self.ijkl)


def sod_uniform(level=5, nsteps=10):
    """Plain 3-D Sod tube on a uniform level (level 5: 32^3 cells, 4096 octs),
    outflow walls, gamma 1.4, CFL 0.8."""
    t = uniform_tree(level)
    return Workload("sod_uniform_l%d" % level, t, sod_state(t, 1.4), 1.4, 0.8, OUTFLOW, nsteps)


def sedov_amr(base=6, lmax=8, radius=0.15, nsteps=50):
    """Sedov blast on a graded tree: base level 6 (64^3 cells) refined to level
    8 where the cell centre is within 0.15 of the box centre; periodic."""
    t = sphere_tree(base, lmax, (0.5, 0.5, 0.5), radius, PERIODIC)
    return Workload("sedov_amr_l%d_l%d" % (base, lmax), t, sedov_state(t, 1.4), 1.4, 0.8, PERIODIC, nsteps)


def random_uniform(level=8, seed=20704, nsteps=20):
    """Uniform periodic box (level 8: 256^3 cells) with lognormal density
    (sigma_ln 0.5), k^-2 random-phase velocities at rms Mach 2, p = 1,
    gamma 5/3."""
    t = uniform_tree(level)
    gam = 5.0 / 3.0
    fields = random_fields_grid(1 << level, seed, gamma=gam)
    u = grid_to_tree_state(t, level, fields, gam)
    return Workload("random_uniform_l%d" % level, t, u, gam, 0.8, PERIODIC, nsteps, {"seed": seed})


def batched_boxes(nbox=64, seed=20704, nsteps=20, base_range=(4, 7), extra_range=(0, 2)):
    """Independent boxes of seeded uneven sizes: base level uniform in
    base_range, 0-2 extra levels on a random sphere; box b mod 3 selects Sod
    (outflow), Sedov (periodic) or random fields (periodic)."""
    boxes = []
    for b in range(nbox):
        rng = np.random.default_rng([seed, 4, b])
        base = int(rng.integers(base_range[0], base_range[1] + 1))
        extra = int(rng.integers(extra_range[0], extra_range[1] + 1))
        centre = rng.uniform(0.2, 0.8, size=3)
        radius = float(rng.uniform(0.1, 0.25))
        kind = b % 3
        if kind == 0:
            bc, gam = OUTFLOW, 1.4
        else:
            bc, gam = PERIODIC, (1.4 if kind == 1 else 5.0 / 3.0)
        if kind == 1:
            centre = np.array([0.5, 0.5, 0.5])   # the blast sits at the box centre
        t = sphere_tree(base, base + extra, centre, radius, bc) if extra else uniform_tree(base)
        if kind == 0:
            u = sod_state(t, gam)
        elif kind == 1:
            u = sedov_state(t, gam)
        else:
            fields = random_fields_grid(1 << base, int(rng.integers(1 << 30)), gamma=gam)
            u = grid_to_tree_state(t, base, fields, gam)
        boxes.append(Workload("box%02d" % b, t, u, gam, 0.8, bc, nsteps,
                              {"base": base, "extra": extra, "kind": ["sod", "sedov", "random"][kind]}))
    return boxes


# Amplitude spread of the clumpy-gas workload's lognormal clumps, bisected
# over [2.5, 2.7] so that the base-7 / level-12 tree with 2000 clumps of seed
# 20705 holds 30 M +- 10 % cells: sigma 2.6 -> 54.4 M, 2.55 -> 20.7 M,
# 2.575 -> 36.3 M, 2.5625 -> 28.1 M cells (3,516,930 octs).
DEEP_AMR_SIGMA_A = 2.5625


def deep_amr(base=7, lmax=12, nclump=2000, seed=20705, sigma_a=None, nsteps=10, radius_level=7):
    """Clumpy gas on a deep cell-by-cell tree: background density 1 plus
    `nclump` seeded Gaussian clumps (lognormal amplitudes, radii 2-20 cells
    of level `radius_level`), at rest, p = rho^(5/3), gamma 5/3, periodic.
    A cell of level base .. lmax-1 is refined where its centre density
    exceeds 8 times the box mean, with the grading closure."""
    sig = DEEP_AMR_SIGMA_A if sigma_a is None else sigma_a
    fld = ClumpField(nclump, seed, sig, radius_level)
    mean = fld.mean()
    ijkl, rho = clump_tree(fld, base, lmax, 8.0 * mean)
    gam = 5.0 / 3.0
    # per-cell density in input order (levels ascending, codes ascending)
    r = np.concatenate([rho[l][1] for l in sorted(rho)]).reshape(-1)
    z = np.zeros_like(r)
    u = conserved(r, z, z, z, r ** gam, gam).reshape(-1, 5)
    u = fill_split_cells(ijkl, u)
    return Workload("deep_amr_l%d_l%d" % (base, lmax), ijkl, u, gam, 0.8, PERIODIC, nsteps,
                    {"sigma_a": sig, "nclump": nclump, "seed": seed, "mean_rho": mean})


def floor_stress(seed=20711, level_base=3, lmax=5, bc=OUTFLOW):
    """A state that drives every density and pressure floor: a refined
    outflow box expanding from its centre (velocity 6 (x - 1/2), density 1)
    at a near-vacuum pressure of 1e-6, with 20 cells emptied (density,
    momentum 0, energy 2.5e-6) and 20 cells whose energy is cut to 0.3 of its
    value, below their kinetic energy; gamma 1.4."""
    t = sphere_tree(level_base, lmax, (0.4, 0.55, 0.5), 0.22, bc)
    cen, _ = cell_centres(t)
    cen = cen.reshape(-1, 3)
    d = cen - 0.5
    rho = np.ones(len(cen))
    vel = 6.0 * d
    u = conserved(rho, vel[:, 0], vel[:, 1], vel[:, 2], np.full(len(cen), 1e-6), 1.4).reshape(-1, 5)
    rng = np.random.default_rng(seed)
    empty = rng.choice(len(u), 20, replace=False)
    u[empty, 0:4] = 0.0
    u[empty, 4] = 2.5e-6
    cut = rng.choice(len(u), 20, replace=False)
    u[cut, 4] = 0.3 * u[cut, 4]
    u = fill_split_cells(t, u)
    return Workload("floor_stress", t, u, 1.4, 0.8, bc, 5, {"seed": seed})
