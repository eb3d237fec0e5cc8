"""ctypes wrapper around oracle.c, the serial FP64 reference (test infrastructure).

Only tests/, the smoke check and the CPU-baseline leg of the benchmark use this
module.  It is independent of the HIP library: it shares no source with it and
never imports the product package.

Layouts (all host numpy arrays, C order):
  ijkl      int32 [n, 4]   oct coordinates (i, j, k) and level l
  u         float64 [8n, 5] conserved state per cell, cell = 8*oct + ix + 2iy + 4iz,
            variables (rho, rho u, rho v, rho w, E)
  nbr27     int32 [n, 27]  neighbour list, entry (dx+1) + 3(dy+1) + 9(dz+1)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

OUTSIDE = -(2 ** 31)
PERIODIC, OUTFLOW = 0, 1
OK, EUNGRADED = 0, 4


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"] + extra + \
          ["-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(force=True):
    """Compile oracle.c with gcc, -O2, no FMA contraction, no fast-math:
    liboracle.so (serial) and liboracle_omp.so (the same source with OpenMP
    over the octs of a level; same bits)."""
    if force or not os.path.exists(_LIB_PATH):
        _compile(_LIB_PATH, [])
    if force or not os.path.exists(_LIB_OMP_PATH):
        _compile(_LIB_OMP_PATH, ["-fopenmp"])
    return _LIB_PATH


_libs = {}
_threads = False


def use_threads(enable):
    """Route the calls of this module to the OpenMP build (True) or the
    serial one (False); returns the previous setting."""
    global _threads
    prev = _threads
    _threads = bool(enable)
    return prev


class threads:
    """Context manager: the OpenMP build inside the block."""

    def __init__(self, enable=True):
        self.enable = enable

    def __enter__(self):
        self.prev = use_threads(self.enable)
        return self

    def __exit__(self, *exc):
        use_threads(self.prev)
        return False


def lib():
    key = _threads
    if key not in _libs:
        path = _LIB_OMP_PATH if key else _LIB_PATH
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, ["-fopenmp"] if key else [])
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32
        L.orc_hilbert.restype = ctypes.c_uint64
        L.orc_hilbert.argtypes = [ctypes.c_int, u32, u32, u32]
        L.orc_key.restype = ctypes.c_uint64
        L.orc_key.argtypes = [i32, i32, i32, i32]
        L.orc_keys.restype = None
        L.orc_keys.argtypes = [i64, P, P]
        L.orc_tree_order.restype = None
        L.orc_tree_order.argtypes = [i64, P, P]
        L.orc_neighbours.restype = ctypes.c_int
        L.orc_neighbours.argtypes = [i64, P, ctypes.c_int, P, P, P, P]
        L.orc_prim.restype = None
        L.orc_prim.argtypes = [P, f64, P]
        L.orc_minmod.restype = f64
        L.orc_minmod.argtypes = [f64, f64]
        L.orc_predict.restype = None
        L.orc_predict.argtypes = [P, P, f64, f64, P]
        L.orc_hllc.restype = None
        L.orc_hllc.argtypes = [P, P, ctypes.c_int, f64, P]
        L.orc_cfl_dt.restype = f64
        L.orc_cfl_dt.argtypes = [i64, P, P, P, f64, f64]
        L.orc_hydro_octs.restype = None
        L.orc_hydro_octs.argtypes = [i64, P, P, P, i64, i64, P, P, P, f64, f64]
        L.orc_step.restype = f64
        L.orc_step.argtypes = [i64, P, P, P, P, P, f64, f64]
        L.orc_step_fixed.restype = f64
        L.orc_step_fixed.argtypes = [i64, P, P, P, P, P, f64, f64]
        L.orc_run.restype = None
        L.orc_run.argtypes = [i64, P, P, P, P, P, f64, f64, i64, P]
        L.orc_cfl_dt_subcycled.restype = f64
        L.orc_cfl_dt_subcycled.argtypes = [i64, P, P, P, f64, f64]
        L.orc_set_ghost_mode.restype = None
        L.orc_set_ghost_mode.argtypes = [ctypes.c_int]
        L.orc_get_ghost_mode.restype = ctypes.c_int
        L.orc_get_ghost_mode.argtypes = []
        L.orc_oct_tile.restype = None
        L.orc_oct_tile.argtypes = [i64, P, P, P, P, i64, P]
        L.orc_mg_vcycles.restype = None
        L.orc_mg_vcycles.argtypes = [ctypes.c_int] * 6 + [P, P, P]
        L.orc_mg_residual.restype = None
        L.orc_mg_residual.argtypes = [ctypes.c_int, P, P, P]
        L.orc_mg_prolong_add.restype = None
        L.orc_mg_prolong_add.argtypes = [ctypes.c_int, P, P]
        L.orc_mg_smooth.restype = None
        L.orc_mg_smooth.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
        L.orc_mg_amr_vcycles.restype = None
        L.orc_mg_amr_vcycles.argtypes = [ctypes.c_int] * 6 + [P, P, P, P, P]
        L.orc_mg_amr_residual.restype = None
        L.orc_mg_amr_residual.argtypes = [ctypes.c_int, P, P, P, P, P]
        L.orc_mg_amr_coarse_sweeps.restype = None
        L.orc_mg_amr_coarse_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int]
        L.orc_mg_amr_masks.restype = None
        L.orc_mg_amr_masks.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        L.orc_refine.restype = ctypes.c_int
        L.orc_refine.argtypes = [i64, P, P, P, ctypes.c_int, f64, f64, ctypes.c_int, ctypes.c_int, P, P, i64, P, P, P]
        L.orc_step_subcycled.restype = f64
        L.orc_step_subcycled.argtypes = [i64, P, P, P, P, P, f64, f64]
        L.orc_oct_face_states.restype = None
        L.orc_oct_face_states.argtypes = [i64, P, P, P, P, i64, f64, f64, P]
        L.orc_threads.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_floor_counts.restype = None
        L.orc_floor_counts.argtypes = [P]
        L.orc_floor_reset.restype = None
        L.orc_floor_reset.argtypes = []
        _libs[key] = L
    return _libs[key]


def nthreads():
    """Threads the active build's parallel loops use (1 when serial)."""
    return int(lib().orc_threads())


def floor_counts():
    """Floor activations since the last floor_reset(): (primitive density,
    primitive pressure, face-state density, face-state pressure)."""
    out = np.zeros(4, dtype=np.int64)
    lib().orc_floor_counts(_p(out))
    return tuple(int(v) for v in out)


def floor_reset():
    lib().orc_floor_reset()


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def hilbert(b, i, j, k):
    """H_b(i, j, k) on the order-20 curve coarsened to 2^b cubes per side."""
    return int(lib().orc_hilbert(int(b), int(i), int(j), int(k)))


def key(i, j, k, l):
    return int(lib().orc_key(int(i), int(j), int(k), int(l)))


def keys(ijkl):
    ijkl = _c(ijkl, np.int32).reshape(-1, 4)
    out = np.empty(len(ijkl), dtype=np.uint64)
    lib().orc_keys(len(ijkl), _p(ijkl), _p(out))
    return out


def tree_order(ijkl):
    """perm such that ijkl[perm] is in key order (level, then Hilbert)."""
    ijkl = _c(ijkl, np.int32).reshape(-1, 4)
    perm = np.empty(len(ijkl), dtype=np.int64)
    lib().orc_tree_order(len(ijkl), _p(ijkl), _p(perm))
    return perm


def neighbours(ijkl, bc):
    """(status, bad_oct, nbr27[n,27], father_cell[n], son_mask[n]) for key-ordered octs."""
    ijkl = _c(ijkl, np.int32).reshape(-1, 4)
    n = len(ijkl)
    nbr = np.zeros((n, 27), dtype=np.int32)
    fc = np.zeros(n, dtype=np.int32)
    sm = np.zeros(n, dtype=np.uint8)
    bad = np.zeros(1, dtype=np.int64)
    st = lib().orc_neighbours(n, _p(ijkl), int(bc), _p(nbr), _p(fc), _p(sm), _p(bad))
    return st, int(bad[0]), nbr, fc, sm


def prim(U, gamma):
    U = _c(U, np.float64)
    W = np.empty(5)
    lib().orc_prim(_p(U), float(gamma), _p(W))
    return W


def minmod(a, b):
    return lib().orc_minmod(float(a), float(b))


def predict(W, dW, h, gamma):
    """Hancock half step W' from W[5], slopes dW[3,5] and h = dt/(2dx)."""
    W = _c(W, np.float64)
    dW = _c(dW, np.float64).reshape(3, 5)
    Wp = np.empty(5)
    lib().orc_predict(_p(W), _p(dW), float(h), float(gamma), _p(Wp))
    return Wp


def hllc(WL, WR, axis, gamma):
    WL = _c(WL, np.float64)
    WR = _c(WR, np.float64)
    F = np.empty(5)
    lib().orc_hllc(_p(WL), _p(WR), int(axis), float(gamma), _p(F))
    return F


def cfl_dt(ijkl, son_mask, u, gamma, cfl):
    ijkl = _c(ijkl, np.int32)
    sm = _c(son_mask, np.uint8)
    u = _c(u, np.float64)
    return lib().orc_cfl_dt(len(sm), _p(ijkl), _p(sm), _p(u), float(gamma), float(cfl))


GHOST_INJECT, GHOST_LINEAR = 0, 1


def set_ghost_mode(mode):
    """Coarse ghost values for the module-level calls: GHOST_INJECT or
    GHOST_LINEAR (minmod-limited linear interpolation)."""
    lib().orc_set_ghost_mode(int(mode))


def hydro_octs(ijkl, nbr27, son_mask, ob, oe, uold, unew, corr, dt, gamma, ghost=GHOST_INJECT):
    """Hydro update of octs [ob, oe) into unew / corr (arrays modified in place)."""
    set_ghost_mode(ghost)
    ijkl = _c(ijkl, np.int32)
    nbr27 = _c(nbr27, np.int32)
    sm = _c(son_mask, np.uint8)
    assert uold.dtype == np.float64 and uold.flags.c_contiguous
    assert unew.dtype == np.float64 and unew.flags.c_contiguous
    assert corr.dtype == np.float64 and corr.flags.c_contiguous
    lib().orc_hydro_octs(len(sm), _p(ijkl), _p(nbr27), _p(sm), int(ob), int(oe), _p(uold), _p(unew),
                         _p(corr), float(dt), float(gamma))


class Tree:
    """A key-ordered tree with the oracle's own neighbour lists; `ghost`
    selects how coarse ghost cells are filled (GHOST_INJECT, GHOST_LINEAR)."""

    def __init__(self, ijkl, bc, ghost=GHOST_INJECT):
        self.ghost = int(ghost)
        ijkl = _c(ijkl, np.int32).reshape(-1, 4)
        self.perm = tree_order(ijkl)
        self.ijkl = np.ascontiguousarray(ijkl[self.perm])
        self.bc = bc
        self.keys = keys(self.ijkl)
        st, bad, self.nbr27, self.father_cell, self.son_mask = neighbours(self.ijkl, bc)
        if st != OK:
            raise ValueError("tree is not graded (oct %d)" % bad)
        self.n = len(self.ijkl)
        lv = self.ijkl[:, 3]
        self.lmin, self.lmax = int(lv.min()), int(lv.max())
        self.level_begin = {l: int(np.searchsorted(lv, l, side="left")) for l in range(self.lmin, self.lmax + 2)}

    def permute_cells(self, u_input_order):
        """Reorder a per-cell array given in input oct order into key order."""
        u = np.asarray(u_input_order).reshape(-1, 8, 5)
        return np.ascontiguousarray(u[self.perm].reshape(-1, 5))

    def cfl_dt(self, u, gamma, cfl):
        return cfl_dt(self.ijkl, self.son_mask, u, gamma, cfl)

    def step(self, u, gamma, cfl):
        """One global-dt step, in place; returns dt."""
        set_ghost_mode(self.ghost)
        assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape == (8 * self.n, 5)
        return lib().orc_step(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.father_cell), _p(self.son_mask),
                              _p(u), float(gamma), float(cfl))

    def step_fixed(self, u, gamma, dt):
        """One step with the given dt, in place."""
        set_ghost_mode(self.ghost)
        assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape == (8 * self.n, 5)
        return lib().orc_step_fixed(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.father_cell),
                                    _p(self.son_mask), _p(u), float(gamma), float(dt))

    def run(self, u, gamma, cfl, nsteps):
        """nsteps steps in place; returns the array of dts."""
        set_ghost_mode(self.ghost)
        assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape == (8 * self.n, 5)
        dts = np.zeros(nsteps)
        lib().orc_run(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.father_cell), _p(self.son_mask),
                      _p(u), float(gamma), float(cfl), int(nsteps), _p(dts))
        return dts

    def cfl_dt_subcycled(self, u, gamma, cfl):
        """Coarse time step of the subcycled scheme."""
        return lib().orc_cfl_dt_subcycled(self.n, _p(self.ijkl), _p(self.son_mask), _p(_c(u, np.float64)),
                                          float(gamma), float(cfl))

    def step_subcycled(self, u, gamma, cfl):
        """One coarse step with level subcycling, in place; returns the coarse dt."""
        set_ghost_mode(self.ghost)
        assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape == (8 * self.n, 5)
        return lib().orc_step_subcycled(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.father_cell),
                                        _p(self.son_mask), _p(u), float(gamma), float(cfl))

    def run_subcycled(self, u, gamma, cfl, nsteps):
        """nsteps coarse subcycled steps in place; returns the coarse dts."""
        return np.array([self.step_subcycled(u, gamma, cfl) for _ in range(nsteps)])

    def refine(self, u, rho_thresh, grad_thresh, lmax_refine, nsubgrid=2):
        """Flags (per oct, key order, criterion + grading closure) and the
        refined / de-refined tree: (flags, new_ijkl, new_u), the new octs in
        emission order (pass new_ijkl to Tree and new_u to its
        permute_cells).  The criterion's own flags (widened to whole octs when
        nsubgrid = 4) are kept in self.last_crit."""
        assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape == (8 * self.n, 5)
        cap = 9 * self.n
        flags = np.zeros(self.n, np.uint8)
        crit = np.zeros(self.n, np.uint8)
        m = ctypes.c_int64(0)
        new_ijkl = np.zeros((cap, 4), np.int32)
        new_u = np.zeros((8 * cap, 5))
        st = lib().orc_refine(self.n, _p(self.ijkl), _p(self.son_mask), _p(u), int(self.bc), float(rho_thresh),
                              float(grad_thresh), int(lmax_refine), int(nsubgrid), _p(crit), _p(flags), cap,
                              ctypes.byref(m),
                              _p(new_ijkl), _p(new_u))
        if st != OK:
            raise ValueError("refine failed with status %d" % st)
        m = m.value
        self.last_crit = crit
        return flags, new_ijkl[:m].copy(), new_u[:8 * m].copy()

    def face_states(self, u, o, dt, gamma):
        """Face states of oct o's update with time step dt:
        [axis][side][z][y][x][var] over tile coordinates -2..3 (the inner
        4^3 written; side 0 the cell's low face, 1 its high face)."""
        set_ghost_mode(self.ghost)
        out = np.zeros((3, 2, 6, 6, 6, 5))
        lib().orc_oct_face_states(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.son_mask), _p(_c(u, np.float64)),
                                  int(o), float(dt), float(gamma), _p(out))
        return out

    def tile(self, u, o):
        """The 6x6x6 tile of oct o, [z][y][x][var] for tile coordinates -2..3."""
        set_ghost_mode(self.ghost)
        t = np.zeros((6, 6, 6, 5))
        lib().orc_oct_tile(self.n, _p(self.ijkl), _p(self.nbr27), _p(self.son_mask), _p(_c(u, np.float64)), int(o),
                           _p(t))
        return t


# ------------------------------------------------------------ multigrid Poisson

def mg_vcycles(phi, f, ncycles, lcoarse=1, nu1=2, nu2=2, ncoarse=50):
    """V-cycles for Lap phi = f on a periodic N^3 grid ([z][y][x], N = 2^L);
    returns (phi after the cycles, RMS residual after each cycle)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64).copy()
    f = np.ascontiguousarray(f, dtype=np.float64)
    N = phi.shape[0]
    L = int(round(np.log2(N)))
    assert phi.shape == (N, N, N) == f.shape and 1 << L == N
    res = np.zeros(ncycles)
    lib().orc_mg_vcycles(L, int(lcoarse), int(nu1), int(nu2), int(ncoarse), int(ncycles), _p(phi), _p(f), _p(res))
    return phi, res


def mg_residual(phi, f):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    L = int(round(np.log2(phi.shape[0])))
    r = np.zeros_like(phi)
    lib().orc_mg_residual(L, _p(phi), _p(f), _p(r))
    return r


def mg_prolong_add(e, phi):
    e = np.ascontiguousarray(e, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64).copy()
    lib().orc_mg_prolong_add(int(round(np.log2(e.shape[0]))), _p(e), _p(phi))
    return phi


def mg_smooth(phi, f, sweeps):
    phi = np.ascontiguousarray(phi, dtype=np.float64).copy()
    f = np.ascontiguousarray(f, dtype=np.float64)
    lib().orc_mg_smooth(int(round(np.log2(phi.shape[0]))), _p(phi), _p(f), int(sweeps))
    return phi


# ------------------------------------------------- multigrid on an AMR tree

def _level_cells(T, level):
    """Dense [z][y][x] indices (flat, N = 2^level) of the cells of level
    `level`'s octs, in key order (cell c = x + 2y + 4z of each oct)."""
    ob, oe = T.level_begin[level], T.level_begin[level + 1]
    ijk = T.ijkl[ob:oe, :3].astype(np.int64)
    N = 1 << level
    q = np.arange(8)
    x = 2 * ijk[:, 0:1] + (q & 1)
    y = 2 * ijk[:, 1:2] + ((q >> 1) & 1)
    z = 2 * ijk[:, 2:3] + (q >> 2)
    return ((z * N + y) * N + x).reshape(-1), 8 * ob, 8 * oe


def _dense_level(T, level, values, fill):
    N = 1 << level
    d = np.full(N ** 3, fill, dtype=np.float64)
    idx, cb, ce = _level_cells(T, level)
    d[idx] = values[cb:ce]
    return d


def mg_amr_level(T, phi, f, level, ncycles, lcoarse=1, nu1=2, nu2=2, ncoarse=50):
    """V-cycles for Lap phi = f on the cells of level `level` of tree T
    (periodic), the coarser level's potential giving the Dirichlet data at
    the level's boundary.  phi and f are per-cell arrays in key order (8
    per oct); phi's entries on level `level` are updated in place (the
    others are read only).  Returns the RMS residual of the level's cells
    after each cycle.  Dense grids: for levels up to about 8."""
    assert T.bc == PERIODIC
    assert phi.dtype == np.float64 and phi.flags.c_contiguous and phi.shape == (8 * T.n,)
    N = 1 << level
    idx, cb, ce = _level_cells(T, level)
    inside = np.zeros(N ** 3, np.uint8)
    inside[idx] = 1
    dphi = np.zeros(N ** 3)
    dphi[idx] = phi[cb:ce]
    df = np.zeros(N ** 3)
    df[idx] = f[cb:ce]
    phic = _dense_level(T, level - 1, phi, np.nan) if level > T.lmin else None
    res = np.zeros(ncycles)
    lib().orc_mg_amr_vcycles(int(level), int(lcoarse), int(nu1), int(nu2), int(ncoarse), int(ncycles), _p(inside),
                             None if phic is None else _p(phic), _p(dphi), _p(df), _p(res))
    phi[cb:ce] = dphi[idx]
    return res


def mg_amr_residual(T, phi, f, level):
    """Residual f - Lap phi of the cells of level `level` (key order)."""
    N = 1 << level
    idx, cb, ce = _level_cells(T, level)
    inside = np.zeros(N ** 3, np.uint8)
    inside[idx] = 1
    dphi = np.zeros(N ** 3)
    dphi[idx] = phi[cb:ce]
    df = np.zeros(N ** 3)
    df[idx] = f[cb:ce]
    phic = _dense_level(T, level - 1, phi, np.nan) if level > T.lmin else None
    r = np.zeros(N ** 3)
    lib().orc_mg_amr_residual(int(level), _p(inside), None if phic is None else _p(phic), _p(dphi), _p(df), _p(r))
    return r[idx]


def mg_amr_masks(T, level, lcoarse=1):
    """The masks of levels lcoarse .. level of level `level`'s V-cycle,
    dense, as a dict level -> [N][N][N]."""
    N = 1 << level
    idx, _, _ = _level_cells(T, level)
    inside = np.zeros(N ** 3, np.uint8)
    inside[idx] = 1
    total = sum(1 << (3 * l) for l in range(lcoarse, level + 1))
    out = np.zeros(total)
    lib().orc_mg_amr_masks(int(level), int(lcoarse), _p(inside), _p(out))
    masks, off = {}, 0
    for l in range(lcoarse, level + 1):
        n = 1 << l
        masks[l] = out[off:off + n ** 3].reshape(n, n, n)
        off += n ** 3
    return masks


def mg_amr_solve(T, f, ncycles, lcoarse=1, nu1=2, nu2=2, ncoarse=50, phi=None):
    """The potential of every level, coarsest first: `ncycles` V-cycles per
    level (f on the coarsest level must have zero mean).  Returns (phi,
    {level: RMS residual after each cycle})."""
    phi = np.zeros(8 * T.n) if phi is None else np.ascontiguousarray(phi, dtype=np.float64).copy()
    res = {}
    for l in range(T.lmin, T.lmax + 1):
        res[l] = mg_amr_level(T, phi, f, l, ncycles, lcoarse, nu1, nu2, ncoarse)
    return phi, res


def mg_amr_coarse_sweeps(inside, m, f, e, sweeps):
    """Gauss-Seidel sweeps of the coarse problem on level m of a V-cycle
    whose finest level's domain is the dense bool grid `inside` (2^L per
    side): Lap e = f, e = 0 on the boundary placed by the masks.  f and e
    are dense over level m; returns the new e."""
    inside = np.ascontiguousarray(inside, dtype=np.uint8).reshape(-1)
    L = int(round(np.log2(round(len(inside) ** (1.0 / 3.0)))))
    assert len(inside) == 1 << (3 * L)
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1).copy()
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    lib().orc_mg_amr_coarse_sweeps(int(L), int(m), _p(inside), _p(f), _p(e), int(sweeps))
    return e


def mg_amr_masks_dense(inside, m):
    """The mask of level m for the dense bool domain grid `inside`."""
    inside = np.ascontiguousarray(inside, dtype=np.uint8).reshape(-1)
    L = int(round(np.log2(round(len(inside) ** (1.0 / 3.0)))))
    total = sum(1 << (3 * l) for l in range(m, L + 1))
    out = np.zeros(total)
    lib().orc_mg_amr_masks(int(L), int(m), _p(inside), _p(out))
    return out[:1 << (3 * m)]
