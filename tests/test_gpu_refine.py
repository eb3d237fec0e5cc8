"""GPU parity of refinement / de-refinement (Sec. 2.2) against the oracle:
flags (criterion alone and closed), the new tree's keys, neighbour lists,
father cells and son masks, and its state, all bit for bit; a dynamic run
(hydro step, then refinement, repeated) against the oracle doing the same;
convergence to the static sphere tree; a full tree reported as RG_EFULL."""
import numpy as np
import pytest
import torch

from gpu_common import parity_metric, say
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu


def _random_amr(seed, bc=I.PERIODIC):
    centre = (0.45, 0.5, 0.55) if bc == I.PERIODIC else (0.2, 0.3, 0.75)
    ijkl = I.sphere_tree(3, 6, centre, 0.2, bc)
    gam = 5.0 / 3.0
    f = I.random_fields_grid(8, seed, gamma=gam)
    return ijkl, bc, I.grid_to_tree_state(ijkl, 3, f, gam), gam


CASES = [
    ("periodic_rho", lambda: _random_amr(51), (1.3, 0.0, 7)),
    ("periodic_grad", lambda: _random_amr(52), (0.0, 0.1, 6)),
    ("outflow_both", lambda: _random_amr(53, I.OUTFLOW), (1.5, 0.15, 7)),
    ("sedov_shrink", lambda: (lambda w: (w.ijkl, w.bc, w.u, w.gamma))(I.sedov_amr(base=4, lmax=6, radius=0.15)),
     (0.0, 0.1, 7)),
]


def _device_tree(ijkl, bc, capacity=None):
    from paper_2607_20704_amd import api
    return api.DeviceTree(ijkl, bc, capacity=capacity)


def _check_tree_equal(D, T2):
    assert D.n == T2.n
    assert np.array_equal(D.keys.cpu().numpy(), T2.keys)
    assert np.array_equal(D.nbr27.cpu().numpy(), T2.nbr27)
    assert np.array_equal(D.father_cell.cpu().numpy(), T2.father_cell)
    assert np.array_equal(D.son_mask.cpu().numpy(), T2.son_mask.astype(np.int32))
    assert (D.lmin, D.lmax) == (T2.lmin, T2.lmax)
    assert all(int(D.level_begin[l]) == T2.level_begin[l] for l in range(T2.lmin, T2.lmax + 2))


@pytest.mark.parametrize("nsubgrid", [2, 4])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_refine_parity(case, nsubgrid):
    name, mk, params = case
    ijkl, bc, u_in, gam = mk()
    say("refine:", name, params, "nsubgrid", nsubgrid)
    T = O.Tree(ijkl, bc)
    D = _device_tree(ijkl, bc, capacity=9 * len(ijkl))
    u = D.to_key_order(u_in)
    ref = T.permute_cells(u_in)
    assert np.array_equal(u.cpu().numpy(), ref)
    flags, ni, nu = T.refine(ref, *params, nsubgrid=nsubgrid)
    got_crit = D.refine_flags(u, *params, closure=False, nsubgrid=nsubgrid).cpu().numpy()
    got_flags = D.refine_flags(u, *params, closure=True, nsubgrid=nsubgrid).cpu().numpy()
    assert np.array_equal(got_crit, T.last_crit.astype(np.int32))
    assert np.array_equal(got_flags, flags.astype(np.int32))
    u2 = D.refine(u, *params, nsubgrid=nsubgrid)
    torch.cuda.synchronize()
    T2 = O.Tree(ni, bc)
    say("  octs %d -> %d, levels %d-%d" % (T.n, T2.n, T2.lmin, T2.lmax))
    _check_tree_equal(D, T2)
    assert np.array_equal(u2.cpu().numpy(), T2.permute_cells(nu))


def test_dynamic_sedov_parity():
    """Sedov blast: hydro step, then refinement on the density jump, ten times;
    the device and the oracle follow the same trees and states."""
    from paper_2607_20704_amd import api
    w = I.sedov_amr(base=4, lmax=6, radius=0.15)
    params = (0.0, 0.08, 7)
    T = O.Tree(w.ijkl, w.bc)
    D = _device_tree(w.ijkl, w.bc, capacity=60000)
    u = D.to_key_order(w.u)
    ref = T.permute_cells(w.u)
    for s in range(10):
        a = torch.empty_like(u)
        dt = D.step(u, a, w.gamma, w.cfl, api.RG_FP64)
        ref_dt = T.step(ref, w.gamma, w.cfl)
        assert float(dt.cpu()[0]) == ref_dt
        flags, ni, nu = T.refine(ref, *params)
        T = O.Tree(ni, w.bc)
        ref = T.permute_cells(nu)
        u = D.refine(a, *params).clone()
        torch.cuda.synchronize()
        say("  step %d: octs %d, levels %d-%d" % (s, T.n, T.lmin, T.lmax))
        _check_tree_equal(D, T)
        worst, dmax = parity_metric(u.cpu().numpy(), ref)
        assert worst <= 1e-12, (s, worst)
    assert T.lmax == 7


def _sphere_state(ijkl, centre, radius):
    cen, _ = I.cell_centres(ijkl)
    d = cen - np.asarray(centre)[None, None, :]
    d = d - np.round(d)
    inside = (d * d).sum(-1) < radius * radius
    z = np.zeros(cen.shape[:2])
    return I.conserved(np.where(inside, 2.0, 1.0), z, z, z, 1.0 + z, 1.4).reshape(-1, 5)


def test_converges_to_static_sphere_tree():
    centre, radius, lmax = (0.4, 0.55, 0.5), 0.22, 6
    D = _device_tree(I.uniform_tree(3), I.PERIODIC, capacity=40000)
    for it in range(2 * lmax):
        n0, keys0 = D.n, D.keys.clone()
        u = torch.as_tensor(np.ascontiguousarray(_sphere_state(D.ijkl_sorted.cpu().numpy(), centre, radius))).cuda()
        D.refine(u, 1.5, 0.0, lmax)
        if D.n == n0 and torch.equal(D.keys, keys0):
            break
    else:
        raise AssertionError("did not converge")
    want = O.Tree(I.sphere_tree(3, lmax, centre, radius, I.PERIODIC), I.PERIODIC)
    assert np.array_equal(D.keys.cpu().numpy(), want.keys)


def test_full_tree_is_reported_and_left_unchanged():
    from paper_2607_20704_amd import api, _lib as L
    ijkl, bc, u_in, gam = _random_amr(54)
    D = _device_tree(ijkl, bc, capacity=len(ijkl) + 8)
    u = D.to_key_order(u_in)
    keys = D.keys.clone()
    with pytest.raises(api.RgError) as e:
        D.refine(u, 1.0, 0.0, 7)
    assert e.value.status == L.RG_EFULL
    assert torch.equal(D.keys, keys)
    # the tree still steps
    T = O.Tree(ijkl, bc)
    a = torch.empty_like(u)
    D.step(u, a, gam, 0.8, api.RG_FP64)
    ref = T.permute_cells(u_in)
    T.step(ref, gam, 0.8)
    assert parity_metric(a.cpu().numpy(), ref)[0] <= 1e-12


def test_schedule_rebuilt_after_refine():
    """A refined tree with its schedule rebuilt steps to the same bits as
    without one."""
    from paper_2607_20704_amd import api
    w = I.sedov_amr(base=5, lmax=6, radius=0.2)
    D = _device_tree(w.ijkl, w.bc, capacity=60000)
    u = D.refine(D.to_key_order(w.u), 0.0, 0.05, 7).clone()
    assert D.sched is not None and sum(c[0] for c in D.schedule_counts().values()) > 0
    a, _ = D.run(u, w.gamma, w.cfl, 3)
    U = api.DeviceTree(D.ijkl_sorted.cpu().numpy(), w.bc, schedule=False)
    b, _ = U.run(u, w.gamma, w.cfl, 3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


SCHED_TREES = [
    ("uniform_l5", lambda: (I.uniform_tree(5), I.PERIODIC)),
    ("sedov_l4_l6", lambda: (I.sedov_amr(base=4, lmax=6).ijkl, I.PERIODIC)),
    ("sphere_5_6_outflow", lambda: (I.sphere_tree(5, 6, (0.3, 0.6, 0.55), 0.2, I.OUTFLOW), I.OUTFLOW)),
    ("deep_amr_l4_l7", lambda: (I.deep_amr(base=4, lmax=7, nclump=60, sigma_a=2.0).ijkl, I.PERIODIC)),
]


@pytest.mark.parametrize("case", SCHED_TREES, ids=[c[0] for c in SCHED_TREES])
def test_device_schedule_equals_host(case):
    from paper_2607_20704_amd import api
    name, mk = case
    ijkl, bc = mk()
    D = api.DeviceTree(ijkl, bc)
    dev = D.schedule_lists()
    D.build_schedule(on_host=True)
    host = D.schedule_lists()
    assert dev.keys() == host.keys()
    for k in dev:
        for a, b in zip(dev[k], host[k]):
            assert np.array_equal(a, b), (name, k)
    say("  %s: bricks %d" % (name, sum(len(v[0]) for k, v in dev.items() if k != "nbr")))


def _leaf_totals_dev(D, u):
    """Leaf sums of volume * U on the device (float64)."""
    lv = D.ijkl_sorted[:, 3].to(torch.float64)
    bits = torch.arange(8, device="cuda", dtype=torch.int32)
    leaf = ((D.son_mask[:, None] >> bits[None, :]) & 1) == 0
    vol = torch.pow(2.0, -3.0 * lv)[:, None] * leaf
    w = vol.reshape(-1, 1)
    return (w * u).sum(0).cpu().numpy(), (w * u.abs()).sum(0).cpu().numpy()


def test_full_deep_amr_refine_properties(deep_full):
    """The 3.5 M-oct clumpy tree refined with the criterion it was built
    with, in the configuration the benchmark times: the new tree is graded,
    kept octs carry their cells unchanged and children exactly where the
    closed flags are, new octs hold their father's values, the criterion's
    flags are among the closed ones, and leaf sums are unchanged."""
    from paper_2607_20704_amd import api, _lib as L
    w = deep_full
    n = len(w.ijkl)
    thr = 8.0 * w.meta["mean_rho"]
    D = api.DeviceTree(w.ijkl, w.bc, capacity=int(1.25 * n))
    u = torch.empty((8 * D.capacity, 5), dtype=torch.float64, device="cuda")
    u[:8 * n] = D.to_key_order(w.u)
    u = u[:8 * n]
    crit = D.refine_flags(u, thr, 0.0, 12, closure=False).cpu().numpy()
    flags = D.refine_flags(u, thr, 0.0, 12, closure=True).cpu().numpy()
    assert np.all((crit & ~flags) == 0) and crit.any()
    tot0, abs0 = _leaf_totals_dev(D, u)
    keys0 = D.keys.cpu().numpy()
    father0 = D.father_cell.cpu().numpy()
    lv0 = D.ijkl_sorted[:, 3].cpu().numpy()
    u_old = u.cpu().numpy().reshape(-1, 8, 5)
    u2 = D.refine(u, thr, 0.0, 12)
    st, bad = api.check_ws(D.hash_ws)
    assert st == L.RG_OK, (st, bad)
    keys1 = D.keys.cpu().numpy()
    ijkl1 = D.ijkl_sorted.cpu().numpy()
    son1 = D.son_mask.cpu().numpy()
    u_new = u2.cpu().numpy().reshape(-1, 8, 5)
    say("  octs %d -> %d" % (n, D.n))
    # kept octs
    kept = lv0 == lv0.min()
    nf = father0 >= 0
    kept[nf] = ((flags[father0[nf] >> 3] >> (father0[nf] & 7)) & 1) == 1
    pos = np.searchsorted(keys1, keys0)
    pos = np.minimum(pos, len(keys1) - 1)
    present = keys1[pos] == keys0
    assert np.array_equal(present, kept)
    assert np.array_equal(u_new[pos[kept]], u_old[kept])
    assert np.array_equal(son1[pos[kept]], flags[kept] & 0xff)
    # new octs: father cell's values in all eight cells
    fresh = np.ones(len(keys1), bool)
    fresh[pos[kept]] = False
    fk = keys1[fresh] >> np.uint64(3)
    fo = np.searchsorted(keys0, fk)
    assert np.array_equal(keys0[fo], fk)
    c = ijkl1[fresh]
    cell = (c[:, 0] & 1) + 2 * (c[:, 1] & 1) + 4 * (c[:, 2] & 1)
    src = u_old[fo, cell]
    assert np.array_equal(u_new[fresh], np.repeat(src[:, None, :], 8, axis=1))
    tot1, abs1 = _leaf_totals_dev(D, u2)
    assert np.all(np.abs(tot1 - tot0) <= 1e-12 * np.maximum(abs0, abs1))


def test_dynamic_subcycled_parity():
    """Subcycled coarse steps with refinement after each one (Sedov blast,
    linear coarse ghosts, 4^3-cell blocks): the device follows the oracle's
    trees, time steps and states bit for bit."""
    from paper_2607_20704_amd import api
    w = I.sedov_amr(base=4, lmax=6, radius=0.15)
    params = (0.0, 0.08, 7)
    T = O.Tree(w.ijkl, w.bc, ghost=O.GHOST_LINEAR)
    D = api.DeviceTree(w.ijkl, w.bc, capacity=60000, ghost=api.L.RG_GHOST_LINEAR)
    ref = T.permute_cells(w.u)
    u = torch.empty((8 * D.capacity, 5), dtype=torch.float64, device="cuda")
    u[:8 * D.n] = D.to_key_order(w.u)
    for s in range(4):
        n8 = 8 * D.n
        dt = D.step_subcycled(u[:n8], w.gamma, w.cfl)
        ref_dt = T.step_subcycled(ref, w.gamma, w.cfl)
        assert float(dt[0].cpu()) == ref_dt
        flags, ni, nu = T.refine(ref, *params, nsubgrid=4)
        T = O.Tree(ni, w.bc, ghost=O.GHOST_LINEAR)
        ref = T.permute_cells(nu)
        u = D.refine(u[:n8], *params, nsubgrid=4).clone()
        u = torch.cat([u, torch.empty((8 * D.capacity - u.shape[0], 5), dtype=torch.float64, device="cuda")])
        torch.cuda.synchronize()
        say("  coarse step %d: octs %d, levels %d-%d" % (s, T.n, T.lmin, T.lmax))
        _check_tree_equal(D, T)
        assert np.array_equal(u[:8 * D.n].cpu().numpy(), ref)
