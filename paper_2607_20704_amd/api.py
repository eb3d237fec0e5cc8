"""Thin Python binding of include/rg.h over PyTorch device tensors.

Functions carry the C names without the ``rg_`` prefix and take torch tensors
on the current HIP device; they marshal pointers, sizes and the current
stream and raise RgError on a non-OK status.  PyTorch supplies device memory
and streams only: every step of the computation runs in librg.so's kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import (RG_BC_OUTFLOW, RG_BC_PERIODIC, RG_FP64, RG_MAX_LEVEL, RG_MIXED, RG_NBR_OUTSIDE,  # noqa: F401
                   RG_STEP_REBUILD, RgError, RgTree, RgTuning, check)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _tuning(tune):
    """tune: None or (octs_per_group, threads[, no_bricks[, persistent[, brick_waves[, no_groups[,
    group_threads[, no_pairs]]]]]])."""
    if tune is None:
        return None
    t = RgTuning()
    t.octs_per_group, t.threads = int(tune[0]), int(tune[1])
    t.no_bricks = int(tune[2]) if len(tune) > 2 else 0
    t.persistent = int(tune[3]) if len(tune) > 3 else 0
    t.brick_waves = int(tune[4]) if len(tune) > 4 else 0
    t.no_groups = int(tune[5]) if len(tune) > 5 else 0
    t.group_threads = int(tune[6]) if len(tune) > 6 else 0
    t.no_pairs = int(tune[7]) if len(tune) > 7 else 0
    return ctypes.byref(t)


def _u8(n):
    return torch.empty(int(n), dtype=torch.uint8, device="cuda")


# ---------------------------------------------------------------- keys, order

def encode_keys(ijkl):
    keys = torch.empty(ijkl.shape[0], dtype=torch.uint64, device="cuda")
    check(L.lib().rg_encode_keys(_ptr(ijkl), ijkl.shape[0], _ptr(keys), _stream()))
    return keys


def decode_keys(keys):
    ijkl = torch.empty((keys.shape[0], 4), dtype=torch.int32, device="cuda")
    check(L.lib().rg_decode_keys(_ptr(keys), keys.shape[0], _ptr(ijkl), _stream()))
    return ijkl


def key_host(i, j, k, l):
    return int(L.lib().rg_key_host(int(i), int(j), int(k), int(l)))


def key_coords_host(key):
    out = (ctypes.c_int32 * 4)()
    L.lib().rg_key_coords_host(ctypes.c_uint64(int(key)), out)
    return tuple(out)


def fnv1a64(key):
    return int(L.lib().rg_fnv1a64(ctypes.c_uint64(int(key))))


def sort_keys(keys):
    n = keys.shape[0]
    ws_bytes = L.lib().rg_sort_workspace_bytes(n)
    ws = _u8(ws_bytes)
    out = torch.empty_like(keys)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    check(L.lib().rg_sort_keys(_ptr(keys), n, _ptr(out), _ptr(perm), _ptr(ws), ws_bytes, _stream()))
    return out, perm


def level_ranges(sorted_keys):
    begin = torch.empty(RG_MAX_LEVEL + 2, dtype=torch.int64, device="cuda")
    check(L.lib().rg_level_ranges(_ptr(sorted_keys), sorted_keys.shape[0], _ptr(begin), _stream()))
    return begin


def permute_rows(x, perm):
    out = torch.empty_like(x)
    rows = perm.shape[0]
    row_doubles = x.numel() // rows if rows else 1   # a row is everything of one permuted item
    check(L.lib().rg_permute_rows(_ptr(x), _ptr(perm), rows, row_doubles, _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------- hash table

def hash_workspace_bytes(n):
    return int(L.lib().rg_hash_workspace_bytes(int(n)))


def hash_build(keys, ws=None):
    n = keys.shape[0]
    nb = hash_workspace_bytes(n)
    if ws is None:
        ws = _u8(nb)
    check(L.lib().rg_hash_build(_ptr(keys), n, _ptr(ws), ws.numel(), _stream()))
    return ws


def hash_build_noalloc(keys, table):
    """Builds the hash table of `keys` into the caller's `table` (uint8,
    256-byte aligned) with the library's static scratch: no allocation."""
    check(L.lib().rg_hash_build_noalloc(_ptr(keys), keys.shape[0], _ptr(table), table.numel(), _stream()))
    return table


def hash_lookup(ws, q):
    out = torch.empty(q.shape[0], dtype=torch.int32, device="cuda")
    check(L.lib().rg_hash_lookup(_ptr(ws), _ptr(q), q.shape[0], _ptr(out), _stream()))
    return out


def check_ws(ws):
    """(status, bad_index) of the device-side flags; synchronises."""
    bad = ctypes.c_int64(-1)
    st = L.lib().rg_check(_ptr(ws), ctypes.byref(bad), _stream())
    return st, bad.value


# ---------------------------------------------------------------- neighbours

def build_neighbours(ws, keys, lmin, bc, nbr27=None, father_cell=None, son_mask=None):
    n = keys.shape[0]
    nbr27 = nbr27 if nbr27 is not None else torch.empty((n, 27), dtype=torch.int32, device="cuda")
    father_cell = father_cell if father_cell is not None else torch.empty(n, dtype=torch.int32, device="cuda")
    son_mask = son_mask if son_mask is not None else torch.empty(n, dtype=torch.int32, device="cuda")
    check(L.lib().rg_build_neighbours(_ptr(ws), _ptr(keys), n, int(lmin), int(bc), _ptr(nbr27), _ptr(father_cell),
                                      _ptr(son_mask), _stream()))
    return nbr27, father_cell, son_mask


# ---------------------------------------------------------------- hydro

def hydro_step_level(dx, dt, gamma, uold, unew, nbr27, son_mask, oct_begin, oct_end, corr=None, corr_base=0,
                     form=RG_FP64, tune=None, cfl=0.0, dt_next=None):
    check(L.lib().rg_hydro_step_level(float(dx), _ptr(dt), float(gamma), _ptr(uold), _ptr(unew), _ptr(nbr27),
                                      _ptr(son_mask), int(oct_begin), int(oct_end), _ptr(corr), int(corr_base),
                                      float(cfl), _ptr(dt_next), int(form), _tuning(tune), _stream()))


def apply_coarse_corrections(unew, corr, corr_base, nbr27, oct_begin, oct_end):
    check(L.lib().rg_apply_coarse_corrections(_ptr(unew), _ptr(corr), int(corr_base), _ptr(nbr27), int(oct_begin),
                                              int(oct_end), _stream()))


def restrict_level(u, father_cell, oct_begin, oct_end):
    check(L.lib().rg_restrict_level(_ptr(u), _ptr(father_cell), int(oct_begin), int(oct_end), _stream()))


def cfl_dt(u, son_mask, level_begin, lmin, lmax, gamma, cfl, dt=None):
    dt = dt if dt is not None else torch.empty(1, dtype=torch.float64, device="cuda")
    lb = np.ascontiguousarray(level_begin, dtype=np.int64)
    check(L.lib().rg_cfl_dt(_ptr(u), _ptr(son_mask), lb.ctypes.data_as(ctypes.c_void_p), int(lmin), int(lmax),
                            float(gamma), float(cfl), _ptr(dt), _stream()))
    return dt


def cfl_dt_corrected(u, nbr27, level_begin, lmin, lmax, gamma, cfl, dt):
    lb = np.ascontiguousarray(level_begin, dtype=np.int64)
    check(L.lib().rg_cfl_dt_corrected(_ptr(u), _ptr(nbr27), lb.ctypes.data_as(ctypes.c_void_p), int(lmin), int(lmax),
                                      float(gamma), float(cfl), _ptr(dt), _stream()))


# ---------------------------------------------------------------- whole tree

class DeviceTree:
    """A tree resident on the device: sorted keys, hash table, neighbour
    lists and the coarse-fine correction buffer, built from oct coordinates
    by the library (encode, radix sort, level ranges, hash, neighbours)."""

    def __init__(self, ijkl, bc, schedule=True, capacity=None, ghost=0):
        ijkl_d = torch.as_tensor(np.ascontiguousarray(ijkl, dtype=np.int32)).to("cuda")
        self.bc = int(bc)
        self.ghost = int(ghost)
        n = int(ijkl_d.shape[0])
        cap = int(capacity) if capacity else n
        if cap < n:
            raise ValueError("capacity %d below the oct count %d" % (cap, n))
        self.capacity = cap
        keys_in = encode_keys(ijkl_d)
        keys, self.perm = sort_keys(keys_in)
        # every per-oct buffer holds `capacity` octs; the attributes below are
        # views of the first n_oct rows (re-cut after a refinement)
        self._keys = torch.empty(cap, dtype=torch.uint64, device="cuda")
        self._keys[:n] = keys
        self.hash_ws = torch.empty(hash_workspace_bytes(cap), dtype=torch.uint8, device="cuda")
        self._nbr27 = torch.empty((cap, 27), dtype=torch.int32, device="cuda")
        self._father_cell = torch.empty(cap, dtype=torch.int32, device="cuda")
        self._son_mask = torch.empty(cap, dtype=torch.int32, device="cuda")
        self._ijkl = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
        self._ijkl[:n] = decode_keys(keys)
        self.keys_scratch = torch.empty(cap, dtype=torch.uint64, device="cuda")
        self.perm_scratch = torch.empty(cap, dtype=torch.int32, device="cuda")
        self.sort_ws = _u8(L.lib().rg_sort_workspace_bytes(cap))
        self.level_begin_dev = torch.empty(RG_MAX_LEVEL + 2, dtype=torch.int64, device="cuda")
        self._set_size(n, level_ranges(keys).cpu().numpy())
        self._corr = None
        if capacity or self.lmax > self.lmin:
            self._corr = torch.empty(cap * 30, dtype=torch.float64, device="cuda")
        self.rebuild()
        st, bad = check_ws(self.hash_ws)
        if st != L.RG_OK:
            raise RgError(st, "tree build failed (%s) at index %d" % (L.lib().rg_status_string(st).decode(), bad))
        self._desc = self._descriptor()
        self.sched = None
        self._want_schedule = schedule
        if schedule:
            self.build_schedule()

    def _set_size(self, n, begin):
        self.n = int(n)
        self.level_begin = np.asarray(begin, dtype=np.int64).copy()
        present = [l for l in range(1, RG_MAX_LEVEL + 1) if self.level_begin[l + 1] > self.level_begin[l]]
        self.lmin, self.lmax = min(present), max(present)
        self.keys = self._keys[:self.n]
        self.nbr27 = self._nbr27[:self.n]
        self.father_cell = self._father_cell[:self.n]
        self.son_mask = self._son_mask[:self.n]
        self.ijkl_sorted = self._ijkl[:self.n]
        self.corr_base = int(self.level_begin[self.lmin + 1])

    @property
    def corr(self):
        """Coarse-fine correction buffer (30 doubles per oct above lmin), or
        None for a single-level tree."""
        if self._corr is None or self.n == self.corr_base:
            return None
        return self._corr

    def build_schedule(self, on_host=False):
        """(Re)build the kernel schedule from the current keys and lists, on
        the device (default) or on the host (rg_schedule_build)."""
        if not hasattr(self, "sched_list") or self.sched_list.numel() < 4 * self.n:
            self.sched_list = torch.empty(4 * self.capacity, dtype=torch.int32, device="cuda")
        self._desc.sched = None
        self.sched = L.RgSchedule()
        if on_host:
            check(L.lib().rg_schedule_build(ctypes.byref(self._desc), _ptr(self.sched_list),
                                            self.sched_list.numel(), ctypes.byref(self.sched), _stream()))
        else:
            if not hasattr(self, "sched_ws"):
                self.sched_ws = _u8(L.lib().rg_schedule_workspace_bytes(self.capacity))
            check(L.lib().rg_schedule_build_device(ctypes.byref(self._desc), _ptr(self.sched_list),
                                                   self.sched_list.numel(), _ptr(self.sched_ws), self.sched_ws.numel(),
                                                   ctypes.byref(self.sched), _stream()))
        self._desc.sched = ctypes.pointer(self.sched)

    def schedule_lists(self):
        """{level: (bricks, per-oct octs, border octs, sibling groups, single
        octs)} as numpy arrays, plus the neighbour-build lists under key
        "nbr"."""
        lst = self.sched_list.cpu().numpy()
        sc = self.sched
        out = {}
        for l in range(self.lmin, self.lmax + 1):
            out[l] = tuple(lst[b:b + c].copy() for b, c in ((sc.brick_begin[l], sc.brick_count[l]),
                                                           (sc.rest_begin[l], sc.rest_count[l]),
                                                           (sc.border_begin[l], sc.border_count[l]),
                                                           (sc.group_begin[l], sc.group_count[l]),
                                                           (sc.single_begin[l], sc.single_count[l])))
        out["nbr"] = (lst[sc.nbr_brick_begin:sc.nbr_brick_begin + sc.nbr_brick_count].copy(),
                      lst[sc.nbr_rest_begin:sc.nbr_rest_begin + sc.nbr_rest_count].copy())
        return out

    def refine(self, u, rho_thresh=0.0, grad_thresh=0.0, lmax=None, out=None, schedule=None, nsubgrid=2):
        """One refinement / de-refinement of the tree from state u (key
        order): the tree is rebuilt in place and the new state, in the new
        key order, is returned (a view of `out`, 8 x capacity x 5 doubles).
        The schedule is rebuilt when the tree was built with one (or when
        schedule=True)."""
        p = L.RgRefineParams()
        p.rho_thresh, p.grad_thresh = float(rho_thresh), float(grad_thresh)
        p.lmax = int(lmax if lmax is not None else self.lmax)
        p.nsubgrid = int(nsubgrid)
        if out is None:
            out = torch.empty((8 * self.capacity, 5), dtype=torch.float64, device="cuda")
        if not hasattr(self, "refine_ws"):
            self.refine_ws = _u8(L.lib().rg_refine_workspace_bytes(self.capacity))
        check(L.lib().rg_refine(ctypes.byref(self._desc), _ptr(u), _ptr(out), ctypes.byref(p), _ptr(self.refine_ws),
                                self.refine_ws.numel(), _stream()))
        d = self._desc
        self._set_size(d.n_oct, [d.level_begin[l] for l in range(RG_MAX_LEVEL + 2)])
        if self._corr is None and self.lmax > self.lmin:
            self._corr = torch.empty(self.capacity * 30, dtype=torch.float64, device="cuda")
            self._desc.d_corr = self._corr.data_ptr()
        self.sched = None
        if schedule if schedule is not None else self._want_schedule:
            self.build_schedule()
        return out[:8 * self.n]

    def refine_flags(self, u, rho_thresh=0.0, grad_thresh=0.0, lmax=None, closure=True, nsubgrid=2):
        """The flags a refinement would act on (uint32 per oct, bit c = cell c)."""
        p = L.RgRefineParams()
        p.rho_thresh, p.grad_thresh = float(rho_thresh), float(grad_thresh)
        p.lmax = int(lmax if lmax is not None else self.lmax)
        p.nsubgrid = int(nsubgrid)
        flags = torch.empty(self.n, dtype=torch.int32, device="cuda")
        check(L.lib().rg_refine_flags(ctypes.byref(self._desc), _ptr(u), ctypes.byref(p), int(bool(closure)),
                                      _ptr(flags), _stream()))
        return flags

    def schedule_counts(self):
        """{level: (bricks, octs outside bricks, sibling groups among them)}
        of the kernel schedule."""
        if self.sched is None:
            return {}
        return {l: (int(self.sched.brick_count[l]), int(self.sched.rest_count[l]), int(self.sched.group_count[l]))
                for l in range(self.lmin, self.lmax + 1)}

    def hydro_level(self, level, dt, gamma, uold, unew, form=RG_FP64, tune=None, cfl=0.0, dt_next=None):
        """The update of one level (scheduled when a schedule exists); with
        dt_next, also folds the new state's CFL limit into it."""
        if self.sched is not None:
            check(L.lib().rg_hydro_step_scheduled(ctypes.byref(self._desc), ctypes.byref(self.sched), int(level),
                                                  _ptr(dt), float(gamma), _ptr(uold), _ptr(unew), float(cfl),
                                                  _ptr(dt_next), int(form), _tuning(tune), _stream()))
        else:
            ob, oe = int(self.level_begin[level]), int(self.level_begin[level + 1])
            hydro_step_level(0.5 ** level, dt, gamma, uold, unew, self.nbr27, self.son_mask, ob, oe,
                             self.corr if level > self.lmin else None, self.corr_base, form, tune, cfl, dt_next)

    def rebuild(self):
        hash_build(self.keys, self.hash_ws)
        build_neighbours(self.hash_ws, self.keys, self.lmin, self.bc, self.nbr27, self.father_cell, self.son_mask)

    def _descriptor(self):
        t = RgTree()
        t.n_oct, t.lmin, t.lmax, t.bc = self.n, self.lmin, self.lmax, self.bc
        t.ghost = self.ghost
        for l in range(RG_MAX_LEVEL + 2):
            t.level_begin[l] = int(self.level_begin[l])
        t.d_keys = self.keys.data_ptr()
        t.d_hash_ws = self.hash_ws.data_ptr()
        t.hash_ws_bytes = self.hash_ws.numel()
        t.d_nbr27 = self.nbr27.data_ptr()
        t.d_father_cell = self.father_cell.data_ptr()
        t.d_son_mask = self.son_mask.data_ptr()
        t.d_corr = self._corr.data_ptr() if self._corr is not None else None
        t.d_ijkl = self.ijkl_sorted.data_ptr()
        t.d_keys_scratch = self.keys_scratch.data_ptr()
        t.d_perm = self.perm_scratch.data_ptr()
        t.d_sort_ws = self.sort_ws.data_ptr()
        t.sort_ws_bytes = self.sort_ws.numel()
        t.d_level_begin = self.level_begin_dev.data_ptr()
        t.capacity = self.capacity
        return t

    def prepare(self, flags=L.RG_STEP_REKEY | RG_STEP_REBUILD):
        """Re-key / re-sort / rebuild hash and neighbour lists on the device."""
        check(L.lib().rg_prepare_tree(ctypes.byref(self._desc), int(flags), _stream()))

    def to_key_order(self, u_input_order):
        """Device copy of a per-cell state given in input oct order, in key order."""
        u = torch.as_tensor(np.ascontiguousarray(u_input_order, dtype=np.float64)).to("cuda")
        return permute_rows(u, self.perm)

    def step(self, uold, unew, gamma, cfl, form=RG_FP64, rebuild=False, dt=None, tune=None, chain=False):
        """One step; rebuild=True re-keys, re-sorts and rebuilds the hash and
        neighbour lists first (the whole tree bookkeeping of a step).  With
        chain=True, dt[0] is this step's time step and the next one is
        written to dt[1] from the new state."""
        dt = dt if dt is not None else torch.empty(2 if chain else 1, dtype=torch.float64, device="cuda")
        flags = (RG_STEP_REBUILD | L.RG_STEP_REKEY) if rebuild else 0
        if chain:
            flags |= L.RG_STEP_CHAIN_DT
        check(L.lib().rg_step(ctypes.byref(self._desc), _ptr(uold), _ptr(unew), float(gamma), float(cfl), int(form),
                              flags, _ptr(dt), _tuning(tune), _stream()))
        return dt

    def run(self, u, gamma, cfl, nsteps, form=RG_FP64, rebuild=False, tune=None, chain=False):
        """nsteps steps; returns (state, dts) with the state in key order.
        With chain=True each step computes the next step's dt inside its
        update (the first one comes from cfl_dt)."""
        a, b = u.clone(), torch.empty_like(u)
        dts = torch.empty(nsteps + 1, dtype=torch.float64, device="cuda")
        if chain:
            cfl_dt(a, self.son_mask, self.level_begin, self.lmin, self.lmax, gamma, cfl, dts[0:1])
        for s in range(nsteps):
            self.step(a, b, gamma, cfl, form, rebuild, dts[s:s + 2] if chain else dts[s:s + 1], tune, chain)
            a, b = b, a
        return a, dts[:nsteps]


    def step_subcycled(self, u, gamma, cfl, form=RG_FP64, rebuild=False, dt=None, tune=None, scratch=None):
        """One coarse step with level subcycling, advancing u in place.
        Returns dt: dt[0] the coarse step, dt[1 + k] level lmin + k's step."""
        if dt is None:
            dt = torch.empty(self.lmax - self.lmin + 2, dtype=torch.float64, device="cuda")
        if scratch is None:
            scratch = torch.empty_like(u)
        if self.corr is not None and getattr(self, "acc", None) is None:
            self.acc = torch.empty_like(self.corr)
        flags = (RG_STEP_REBUILD | L.RG_STEP_REKEY) if rebuild else 0
        check(L.lib().rg_step_subcycled(ctypes.byref(self._desc), _ptr(u), _ptr(scratch),
                                        _ptr(self.acc if self.corr is not None else None), float(gamma), float(cfl),
                                        int(form), flags, _ptr(dt), _tuning(tune), _stream()))
        return dt

    def capture_subcycled(self, u, gamma, cfl, nsteps=1, form=RG_FP64, tune=None):
        """A captured HIP graph of `nsteps` subcycled coarse steps advancing
        u in place (for trees small enough that launching the level
        recursion costs more than the work).  Returns a CapturedSteps that
        owns the graph together with every buffer the graph reads or writes
        (u, the scratch state, the flux accumulator, dts); each replay() runs
        the steps and writes dts[s] (coarse step s's time steps).  The tree
        must not change while the graph is used."""
        nlev = self.lmax - self.lmin + 2
        dts = torch.empty((nsteps, nlev), dtype=torch.float64, device="cuda")
        scratch = torch.empty_like(u)
        if self.corr is not None and getattr(self, "acc", None) is None:
            self.acc = torch.empty_like(self.corr)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for k in range(nsteps):
                self.step_subcycled(u, gamma, cfl, form, False, dts[k], tune, scratch)
        torch.cuda.current_stream().wait_stream(side)
        return CapturedSteps(g, dts, (u, scratch, getattr(self, "acc", None), self))

    def run_subcycled(self, u, gamma, cfl, nsteps, form=RG_FP64, rebuild=False, tune=None):
        """nsteps coarse subcycled steps on a copy of u; returns (state, dts)
        with dts[s] the coarse step of step s."""
        a, scratch = u.clone(), torch.empty_like(u)
        dts = torch.empty((nsteps, self.lmax - self.lmin + 2), dtype=torch.float64, device="cuda")
        for s in range(nsteps):
            self.step_subcycled(a, gamma, cfl, form, rebuild, dts[s], tune, scratch)
        return a, dts[:, 0]


# ---------------------------------------------------------------- multigrid

class CapturedSteps:
    """A captured graph and the device buffers it uses: the buffers live as
    long as this object, so a replay never writes memory the allocator has
    handed out again."""

    def __init__(self, graph, dts, buffers):
        self.graph = graph
        self.dts = dts
        self._buffers = buffers

    def replay(self):
        self.graph.replay()


class Multigrid:
    """Multigrid Poisson V-cycles (rg_mg_vcycles) on a periodic unigrid of
    level `lfine`: the hierarchy is the complete tree of levels 1..lfine,
    built once on the device (keys, hash, neighbour lists)."""

    def __init__(self, lfine, lcoarse=1):
        from . import inputs
        self.lfine, self.lcoarse = int(lfine), int(lcoarse)
        self.tree = DeviceTree(inputs.full_tree(self.lfine), 0, schedule=False)
        n8 = 8 * self.tree.n
        self.phi = torch.zeros((n8,), dtype=torch.float64, device="cuda")
        self.f = torch.zeros_like(self.phi)
        self.r = torch.zeros_like(self.phi)
        lb = self.tree.level_begin
        self.fine = slice(8 * int(lb[self.lfine]), 8 * int(lb[self.lfine + 1]))

    def fine_cells_ijk(self):
        """[m, 3] global cell coordinates of the fine level's cells, in array order."""
        ijkl = self.tree.ijkl_sorted[int(self.tree.level_begin[self.lfine]):].cpu().numpy()
        c = np.arange(8)
        out = np.empty((len(ijkl), 8, 3), np.int64)
        out[..., 0] = 2 * ijkl[:, :1] + (c & 1)
        out[..., 1] = 2 * ijkl[:, 1:2] + ((c >> 1) & 1)
        out[..., 2] = 2 * ijkl[:, 2:3] + (c >> 2)
        return out.reshape(-1, 3)

    def vcycles(self, ncycles, nu1=2, nu2=2, ncoarse=50):
        check(L.lib().rg_mg_vcycles(ctypes.byref(self.tree._desc), _ptr(self.phi), _ptr(self.f), _ptr(self.r),
                                    self.lfine, self.lcoarse, int(nu1), int(nu2), int(ncoarse), int(ncycles),
                                    _stream()))

    def residual(self):
        check(L.lib().rg_mg_residual(ctypes.byref(self.tree._desc), _ptr(self.phi), _ptr(self.f), _ptr(self.r),
                                     self.lfine, _stream()))
        return self.r[self.fine]


class MgLevel:
    """The multigrid hierarchy of one level of a periodic AMR tree
    (rg_mg_level_create): V-cycles for Lap phi = f on the level's cells, the
    coarser level's potential giving the boundary values.  phi and f are
    per-cell arrays over the whole tree (8 n_oct doubles, key order)."""

    def __init__(self, tree, level, lcoarse=1):
        self.tree, self.level = tree, int(level)
        h = ctypes.c_void_p()
        check(L.lib().rg_mg_level_create(ctypes.byref(tree._desc), self.level, int(lcoarse), ctypes.byref(h),
                                         _stream()))
        self._h = h

    def counts(self):
        """{level: octs} of the hierarchy (this level's own octs included)."""
        out = (ctypes.c_int64 * (RG_MAX_LEVEL + 1))()
        check(L.lib().rg_mg_level_counts(self._h, out))
        return {m: int(out[m]) for m in range(RG_MAX_LEVEL + 1) if out[m]}

    def vcycles(self, phi, f, ncycles, nu1=2, nu2=2, ncoarse=50):
        check(L.lib().rg_mg_level_vcycles(self._h, ctypes.byref(self.tree._desc), _ptr(phi), _ptr(f), int(nu1),
                                          int(nu2), int(ncoarse), int(ncycles), _stream()))

    def residual(self, phi, f, r=None):
        """f - Lap phi on this level's cells, as a slice of a per-cell array."""
        r = torch.zeros_like(phi) if r is None else r
        check(L.lib().rg_mg_level_residual(self._h, ctypes.byref(self.tree._desc), _ptr(phi), _ptr(f), _ptr(r),
                                           _stream()))
        lb = self.tree.level_begin
        return r[8 * int(lb[self.level]):8 * int(lb[self.level + 1])]

    def close(self):
        if getattr(self, "_h", None):
            L.lib().rg_mg_level_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mg_solve_levels(tree, f, ncycles, nu1=2, nu2=2, ncoarse=50, lcoarse=1, phi=None, levels=None):
    """The potential of every level of `tree`, coarsest first, `ncycles`
    V-cycles each (f on the coarsest level must have zero mean).  Returns
    (phi, {level: MgLevel}); the hierarchies can be reused while the tree is
    unchanged."""
    phi = torch.zeros_like(f) if phi is None else phi
    levels = levels or {}
    for l in range(tree.lmin, tree.lmax + 1):
        if l not in levels:
            levels[l] = MgLevel(tree, l, lcoarse)
        levels[l].vcycles(phi, f, ncycles, nu1, nu2, ncoarse)
    return phi, levels


# ---------------------------------------------------------------- many trees

class Batch:
    """Independent trees advanced together: every phase of a step is one
    kernel over a work list spanning all trees, and all `nsteps` steps are one
    captured graph (rg_batch_create / rg_batch_run).  Each tree keeps its own
    time step.  `states` are key-ordered device states (copied); after a run
    the result is in `state(t)`, and with an even `nsteps` a further run()
    continues from it."""

    def __init__(self, trees, states, gammas, cfls, nsteps, form=RG_FP64, rebuild=False, tune=None):
        if len(trees) == 0 or not (len(trees) == len(states) == len(gammas) == len(cfls)):
            raise ValueError("trees, states, gammas and cfls must be non-empty lists of one length")
        for t in trees:
            if t.sched is None:
                raise ValueError("every tree needs a schedule (DeviceTree(..., schedule=True))")
        self.trees = list(trees)
        self.nsteps = int(nsteps)
        self.u = [[s.clone() for s in states], [torch.empty_like(s) for s in states]]
        self.dt = torch.empty((self.nsteps + 1) * len(trees), dtype=torch.float64, device="cuda")
        arr = (L.RgBatchTree * len(trees))()
        for k, t in enumerate(trees):
            arr[k].tree = ctypes.pointer(t._desc)
            arr[k].d_u0 = self.u[0][k].data_ptr()
            arr[k].d_u1 = self.u[1][k].data_ptr()
            arr[k].gamma = float(gammas[k])
            arr[k].cfl = float(cfls[k])
        self._h = ctypes.c_void_p()
        flags = RG_STEP_REBUILD if rebuild else 0
        check(L.lib().rg_batch_create(arr, len(trees), int(form), self.nsteps, flags, _tuning(tune), _ptr(self.dt),
                                      _stream(), ctypes.byref(self._h)))

    def run(self):
        check(L.lib().rg_batch_run(self._h, _stream()))

    def state(self, t):
        """State of tree t after the last run (key order)."""
        return self.u[self.nsteps % 2][t]

    def dts(self):
        """Time steps of the last run, [nsteps, ntree]."""
        return self.dt.view(self.nsteps + 1, len(self.trees))[:self.nsteps]

    def close(self):
        if getattr(self, "_h", None):
            L.lib().rg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
