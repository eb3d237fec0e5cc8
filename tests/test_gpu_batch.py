"""The batched form (many trees, one captured graph) against each tree run
alone through rg_step, and against the FP64 oracle.

Bars: bit-identical state and time steps per tree against rg_step on the
tree alone (same form, same kernels per item), for every tuning the batched
form accepts; FP64 state within the parity bar of the oracle."""
import numpy as np
import pytest
import torch

from gpu_common import parity_metric, say
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu

# (octs_per_group, threads, no_bricks, persistent[, brick_waves, no_groups])
BATCH_TUNINGS = [(4, 256, 0, 0), (4, 256, 0, 1), (2, 256, 0, 0), (8, 256, 0, 1), (4, 256, 1, 0),
                 (4, 256, 0, 1, 0, 1)]


def small_boxes(nsteps):
    """Nine seeded boxes: uniform and refined, Sod/Sedov/random, levels 3-7."""
    return I.batched_boxes(nbox=9, seed=20704, nsteps=nsteps, base_range=(3, 5), extra_range=(0, 2))


def device_trees(boxes):
    from paper_2607_20704_amd import api
    trees = [api.DeviceTree(b.ijkl, b.bc) for b in boxes]
    states = [D.to_key_order(b.u.reshape(-1, 5)) for D, b in zip(trees, boxes)]
    torch.cuda.synchronize()
    return trees, states


def alone(D, u0, box, nsteps, form, rebuild):
    u, dts = D.run(u0, box.gamma, box.cfl, nsteps, form=form, rebuild=rebuild)
    torch.cuda.synchronize()
    return u.cpu().numpy(), dts.cpu().numpy()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("tune", BATCH_TUNINGS, ids=["g%d_nb%d_p%d_ng%d" % (t[0], t[2], t[3], t[5] if len(t) > 5 else 0)
                                                     for t in BATCH_TUNINGS])
def test_batch_equals_alone(form, tune):
    from paper_2607_20704_amd import api
    nsteps = 4
    boxes = small_boxes(nsteps)
    say("batch vs alone:", form, tune, "boxes", len(boxes), "octs", [len(b.ijkl) for b in boxes])
    trees, states = device_trees(boxes)
    f = api.RG_FP64 if form == "fp64" else api.RG_MIXED
    B = api.Batch(trees, states, [b.gamma for b in boxes], [b.cfl for b in boxes], nsteps, form=f, tune=tune)
    B.run()
    torch.cuda.synchronize()
    dts = B.dts().cpu().numpy()
    for k, (D, u0, box) in enumerate(zip(trees, states, boxes)):
        want, want_dt = alone(D, u0, box, nsteps, f, rebuild=False)
        got = B.state(k).cpu().numpy()
        assert np.array_equal(dts[:, k], want_dt), (box.name, dts[:, k], want_dt)
        assert np.array_equal(got, want), (box.name, np.abs(got - want).max())
    B.close()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_batch_rebuild_and_repeat(form):
    """With the hash and neighbour rebuild inside the graph, and two runs of
    the graph back to back (continuing from the first run's result)."""
    from paper_2607_20704_amd import api
    nsteps = 2
    boxes = small_boxes(nsteps)
    say("batch rebuild + repeat:", form)
    trees, states = device_trees(boxes)
    f = api.RG_FP64 if form == "fp64" else api.RG_MIXED
    B = api.Batch(trees, states, [b.gamma for b in boxes], [b.cfl for b in boxes], nsteps, form=f, rebuild=True)
    B.run()
    dts1 = B.dts().cpu().numpy().copy()
    B.run()
    torch.cuda.synchronize()
    dts2 = B.dts().cpu().numpy()
    for k, (D, u0, box) in enumerate(zip(trees, states, boxes)):
        want, want_dt = alone(D, u0, box, 2 * nsteps, f, rebuild=True)
        assert np.array_equal(np.concatenate([dts1[:, k], dts2[:, k]]), want_dt), box.name
        assert np.array_equal(B.state(k).cpu().numpy(), want), box.name
        st, bad = api.check_ws(D.hash_ws)
        assert st == api.L.RG_OK, (box.name, st, bad)
    B.close()


def test_batch_fp64_matches_oracle():
    from paper_2607_20704_amd import api
    nsteps = 3
    boxes = small_boxes(nsteps)
    say("batch fp64 vs oracle")
    trees, states = device_trees(boxes)
    B = api.Batch(trees, states, [b.gamma for b in boxes], [b.cfl for b in boxes], nsteps, form=api.RG_FP64)
    B.run()
    torch.cuda.synchronize()
    dts = B.dts().cpu().numpy()
    for k, box in enumerate(boxes):
        T = O.Tree(box.ijkl, box.bc)
        ref = T.permute_cells(box.u.reshape(-1, 5))
        ref_dts = T.run(ref, box.gamma, box.cfl, nsteps)
        worst, dmax = parity_metric(B.state(k).cpu().numpy(), ref)
        say("  %s worst ratio %.3g max |diff| %.3g" % (box.name, worst, dmax))
        assert worst <= 1e-12, box.name
        assert np.all(np.abs(dts[:, k] - ref_dts) <= 1e-12 * ref_dts), box.name
    B.close()


def test_batch_argument_errors():
    from paper_2607_20704_amd import api
    boxes = small_boxes(2)[:2]
    trees, states = device_trees(boxes)
    with pytest.raises(api.RgError):
        api.Batch(trees, states, [b.gamma for b in boxes], [b.cfl for b in boxes], 2, tune=(3, 256))
    with pytest.raises(api.RgError):
        api.Batch(trees, states, [0.5, 1.4], [b.cfl for b in boxes], 2)
    no_sched = api.DeviceTree(boxes[0].ijkl, boxes[0].bc, schedule=False)
    with pytest.raises(ValueError):
        api.Batch([no_sched], states[:1], [1.4], [0.8], 2)
