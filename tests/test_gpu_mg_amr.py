"""GPU parity of the level-by-level multigrid on AMR trees (rg_mg_level_*)
against the oracle's dense solver: bit for bit, level after level.

- Two- and three-level trees (a refined patch inside the box, one wrapping
  across the periodic boundary), coarsest MG level 1 or 2, and the case
  lcoarse == level (sweeps only).
- The Sedov blast tree (base 6, refined to level 8): every level solved in
  turn, 4 V-cycles each; the residual falls by at least 5x per cycle.
- The coarsest level of a tree (complete, periodic) gives the periodic
  solver's values.
- Refused on the host: an outflow tree, a level outside the tree, a handle
  used with another tree."""
import numpy as np
import pytest
import torch

from gpu_common import say
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu


def _api():
    from paper_2607_20704_amd import api
    return api


def _rhs(T, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(8 * T.n)
    cb, ce = 8 * T.level_begin[T.lmin], 8 * T.level_begin[T.lmin + 1]
    f[cb:ce] -= f[cb:ce].mean()
    return f


def _both(ijkl):
    api = _api()
    T = O.Tree(ijkl, I.PERIODIC)
    D = api.DeviceTree(ijkl, I.PERIODIC)
    assert np.array_equal(D.keys.cpu().numpy(), T.keys)
    return T, D


TREES = [
    ("patch_4_5", lambda: I.sphere_tree(4, 5, (0.5, 0.45, 0.55), 0.2, I.PERIODIC), 1),
    ("wrap_4_6", lambda: I.sphere_tree(4, 6, (0.06, 0.9, 0.5), 0.2, I.PERIODIC), 1),
    ("wrap_4_6_lc2", lambda: I.sphere_tree(4, 6, (0.06, 0.9, 0.5), 0.2, I.PERIODIC), 2),
    ("uniform_5", lambda: I.uniform_tree(5), 1),
]


@pytest.mark.parametrize("name,mk,lcoarse", TREES, ids=[t[0] for t in TREES])
def test_levels_bit_exact(name, mk, lcoarse):
    api = _api()
    T, D = _both(mk())
    f = _rhs(T, 3)
    say("level multigrid:", name, T.n, "octs, levels", T.lmin, T.lmax, "lcoarse", lcoarse)
    ref, _ = O.mg_amr_solve(T, f, 3, lcoarse=lcoarse)
    fd = torch.as_tensor(f).cuda()
    phi, levels = api.mg_solve_levels(D, fd, 3, lcoarse=lcoarse)
    got = phi.cpu().numpy()
    for l in range(T.lmin, T.lmax + 1):
        cb, ce = 8 * T.level_begin[l], 8 * T.level_begin[l + 1]
        assert np.array_equal(got[cb:ce], ref[cb:ce]), (l, np.abs(got[cb:ce] - ref[cb:ce]).max())
        r = levels[l].residual(phi, fd).cpu().numpy()
        assert np.array_equal(r, O.mg_amr_residual(T, ref, f, l)), l
    for h in levels.values():
        h.close()


def test_sweeps_only_when_lcoarse_is_the_level():
    api = _api()
    T, D = _both(I.sphere_tree(4, 5, (0.3, 0.6, 0.4), 0.2, I.PERIODIC))
    f = _rhs(T, 5)
    ref = np.zeros(8 * T.n)
    O.mg_amr_level(T, ref, f, 4, 2)
    O.mg_amr_level(T, ref, f, 5, 1, lcoarse=5, ncoarse=7)
    fd = torch.as_tensor(f).cuda()
    phi = torch.zeros_like(fd)
    h4 = api.MgLevel(D, 4)
    h4.vcycles(phi, fd, 2)
    h5 = api.MgLevel(D, 5, lcoarse=5)
    assert h5.counts() == {5: int(T.level_begin[6] - T.level_begin[5])}
    h5.vcycles(phi, fd, 1, ncoarse=7)
    assert np.array_equal(phi.cpu().numpy(), ref)
    h4.close()
    h5.close()


def test_sedov_tree_levels_and_rate():
    api = _api()
    w = I.sedov_amr()
    T, D = _both(w.ijkl)
    f = _rhs(T, 7)
    say("sedov tree: oracle, 3 levels x 4 V-cycles")
    ref, ref_res = O.mg_amr_solve(T, f, 4)
    fd = torch.as_tensor(f).cuda()
    phi = torch.zeros_like(fd)
    for l in range(T.lmin, T.lmax + 1):
        h = api.MgLevel(D, l)
        say("  level", l, "hierarchy", h.counts())
        res = []
        for c in range(4):
            h.vcycles(phi, fd, 1)
            r = h.residual(phi, fd)
            res.append(float(torch.sqrt((r * r).mean())))
        cb, ce = 8 * T.level_begin[l], 8 * T.level_begin[l + 1]
        got = phi[cb:ce].cpu().numpy()
        assert np.array_equal(got, ref[cb:ce]), l
        assert np.allclose(res, ref_res[l], rtol=1e-10), (res, ref_res[l])
        rate = (res[-1] / res[0]) ** (1.0 / 3.0)
        say("  residual", res, "factor per cycle %.3f" % rate)
        assert rate <= 0.2
        h.close()


def test_host_checks():
    api = _api()
    ijkl = I.sphere_tree(3, 4, (0.4, 0.5, 0.5), 0.25, I.OUTFLOW)
    Dout = api.DeviceTree(ijkl, I.OUTFLOW)
    with pytest.raises(api.RgError) as e:
        api.MgLevel(Dout, 4)
    assert e.value.status == api.L.RG_EINVAL
    D = api.DeviceTree(I.sphere_tree(3, 4, (0.4, 0.5, 0.5), 0.25, I.PERIODIC), I.PERIODIC)
    for level, lc in ((2, 1), (5, 1), (4, 0), (4, 5)):
        with pytest.raises(api.RgError) as e:
            api.MgLevel(D, level, lc)
        assert e.value.status == api.L.RG_EINVAL
    h = api.MgLevel(D, 4)
    other = api.DeviceTree(I.sphere_tree(3, 4, (0.6, 0.5, 0.5), 0.2, I.PERIODIC), I.PERIODIC)
    assert other.n != D.n
    phi = torch.zeros(8 * other.n, dtype=torch.float64, device="cuda")
    with pytest.raises(api.RgError) as e:
        h.tree = other
        h.vcycles(phi, phi, 1)
    assert e.value.status == api.L.RG_EINVAL
    h.close()
