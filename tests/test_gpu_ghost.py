"""GPU parity with linearly interpolated coarse ghost cells (minmod-limited,
per tree: rg_tree.ghost = RG_GHOST_LINEAR) against the oracle in the same
mode: global steps, subcycled steps (a four-level tree, where a coarse
ghost cell's neighbours can sit two levels down), the mixed form, kernel
variants and the batched form."""
import numpy as np
import pytest
import torch

from gpu_common import l1_rel, leaf_and_volume, parity_metric, say, small_trees
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu


def _both(ijkl, bc, **kw):
    from paper_2607_20704_amd import api
    T = O.Tree(ijkl, bc, ghost=O.GHOST_LINEAR)
    D = api.DeviceTree(ijkl, bc, ghost=api.L.RG_GHOST_LINEAR, **kw)
    assert np.array_equal(D.keys.cpu().numpy(), T.keys)
    return T, D


AMR_CASES = [c for c in small_trees() if c[0].startswith("amr")]


@pytest.mark.parametrize("case", AMR_CASES, ids=[c[0] for c in AMR_CASES])
def test_fp64_parity_linear_ghosts(case):
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = case
    u_in, gam = mk(ijkl)
    T, D = _both(ijkl, bc)
    u, dts = D.run(D.to_key_order(u_in), gam, 0.8, 10, form=api.RG_FP64)
    torch.cuda.synchronize()
    ref = T.permute_cells(u_in)
    ref_dts = T.run(ref, gam, 0.8, 10)
    worst, dmax = parity_metric(u.cpu().numpy(), ref)
    say("linear ghosts %s: worst %.3g bit-equal %s" % (name, worst, np.array_equal(u.cpu().numpy(), ref)))
    assert worst <= 1e-12
    assert np.array_equal(dts.cpu().numpy(), ref_dts)
    # the injection tree differs: the mode is really applied
    Dinj = api.DeviceTree(ijkl, bc)
    v, _ = Dinj.run(Dinj.to_key_order(u_in), gam, 0.8, 10, form=api.RG_FP64)
    assert not torch.equal(u, v)


def test_subcycled_parity_linear_ghosts():
    from paper_2607_20704_amd import api
    w = I.deep_amr(base=4, lmax=7, nclump=60, sigma_a=2.0)
    T, D = _both(w.ijkl, w.bc)
    u, dts = D.run_subcycled(D.to_key_order(w.u), w.gamma, w.cfl, 3, form=api.RG_FP64)
    torch.cuda.synchronize()
    ref = T.permute_cells(w.u)
    ref_dts = T.run_subcycled(ref, w.gamma, w.cfl, 3)
    worst, dmax = parity_metric(u.cpu().numpy(), ref)
    say("subcycled linear ghosts: worst %.3g" % worst)
    assert np.array_equal(dts.cpu().numpy(), ref_dts)
    assert worst <= 1e-12


def test_mixed_l1_linear_ghosts():
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = AMR_CASES[0]
    u_in, gam = mk(ijkl)
    T, D = _both(ijkl, bc)
    u, _ = D.run(D.to_key_order(u_in), gam, 0.8, 10, form=api.RG_MIXED)
    torch.cuda.synchronize()
    ref = T.permute_cells(u_in)
    T.run(ref, gam, 0.8, 10)
    leaf, vol = leaf_and_volume(T)
    l1 = l1_rel(u.cpu().numpy(), ref, leaf, vol)
    say("mixed linear ghosts L1", l1)
    assert np.all(l1 <= 1e-5)


def test_variants_and_batch_linear_ghosts():
    from paper_2607_20704_amd import api
    w = I.sedov_amr(base=4, lmax=6, radius=0.2)
    T, D = _both(w.ijkl, w.bc)
    u0 = D.to_key_order(w.u)
    base, _ = D.run(u0, w.gamma, w.cfl, 4)
    for tune in [(2, 128), (8, 256), (4, 256, 1), (4, 256, 0, 0, 0, 1)]:
        other, _ = D.run(u0, w.gamma, w.cfl, 4, tune=tune)
        assert torch.equal(base, other), tune
    U = api.DeviceTree(w.ijkl, w.bc, schedule=False, ghost=api.L.RG_GHOST_LINEAR)
    other, _ = U.run(U.to_key_order(w.u), w.gamma, w.cfl, 4)
    assert torch.equal(base, other)
    B = api.Batch([D], [u0], [w.gamma], [w.cfl], 4)
    B.run()
    torch.cuda.synchronize()
    assert torch.equal(B.state(0), base)
    B.close()
