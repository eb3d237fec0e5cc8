"""GPU parity of the hydro path (CFL dt, per-level MUSCL-Hancock/HLLC update,
coarse-fine correction, restriction) against the FP64 oracle.

Bars: dt and integer data bit-exact; FP64 state within 1e-12 per cell
(density and energy relative to the cell value, momenta relative to the
field's largest magnitude); the mixed form within an L1 error of 1e-5 per
conserved field against the FP64 oracle, and conserving mass, momentum and
energy to double rounding."""
import numpy as np
import pytest
import torch

from gpu_common import build_both, l1_rel, leaf_and_volume, parity_metric, say, small_trees
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu

TUNINGS = [(4, 256), (2, 128), (8, 256), (7, 256), (3, 128), (4, 256, 1)]


def device_state(D, u_input):
    return D.to_key_order(u_input.reshape(-1, 5))


def run_device(D, u0, gamma, cfl, nsteps, form, tune=None, rebuild=False):
    from paper_2607_20704_amd import api
    u, dts = D.run(u0, gamma, cfl, nsteps, form=form, tune=tune, rebuild=rebuild)
    torch.cuda.synchronize()
    return u.cpu().numpy(), dts.cpu().numpy()


@pytest.mark.parametrize("case", small_trees(), ids=[c[0] for c in small_trees()])
def test_cfl_dt_bit_exact(case):
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = case
    u_in, gam = mk(ijkl)
    say("dt:", name)
    T, D = build_both(ijkl, bc)
    u = device_state(D, u_in)
    dt = api.cfl_dt(u, D.son_mask, D.level_begin, D.lmin, D.lmax, gam, 0.8).cpu().numpy()[0]
    want = T.cfl_dt(T.permute_cells(u_in), gam, 0.8)
    assert dt == want, (dt, want)


@pytest.mark.parametrize("case", small_trees(), ids=[c[0] for c in small_trees()])
def test_fp64_step_parity(case):
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = case
    u_in, gam = mk(ijkl)
    nsteps = 10
    say("fp64 parity:", name, "steps", nsteps)
    T, D = build_both(ijkl, bc)
    got, dts = run_device(D, device_state(D, u_in), gam, 0.8, nsteps, api.RG_FP64)
    ref = T.permute_cells(u_in)
    ref_dts = T.run(ref, gam, 0.8, nsteps)
    worst, dmax = parity_metric(got, ref)
    say("  worst ratio %.3g, max |diff| %.3g, dt diff %.3g" % (worst, dmax, np.abs(dts - ref_dts).max()))
    assert worst <= 1e-12
    assert np.all(np.abs(dts - ref_dts) <= 1e-12 * ref_dts)


def test_fp64_sod_config_parity():
    """Plain 3-D Sod tube, level 5 (32^3 cells, 4096 octs), outflow, 10 steps."""
    from paper_2607_20704_amd import api
    w = I.sod_uniform()
    say("fp64 parity: sod 32^3, 10 steps")
    T, D = build_both(w.ijkl, w.bc)
    got, dts = run_device(D, device_state(D, w.u), w.gamma, w.cfl, w.nsteps, api.RG_FP64)
    ref = T.permute_cells(w.u)
    ref_dts = T.run(ref, w.gamma, w.cfl, w.nsteps)
    worst, dmax = parity_metric(got, ref)
    say("  worst ratio %.3g, max |diff| %.3g" % (worst, dmax))
    assert worst <= 1e-12
    assert np.array_equal(dts, ref_dts) or np.all(np.abs(dts - ref_dts) <= 1e-12 * ref_dts)


@pytest.mark.parametrize("nsteps", [10, 50])
def test_fp64_sedov_amr_config_parity(nsteps):
    """Sedov blast on the graded base-6 / level-8 tree (67,344 octs), periodic."""
    from paper_2607_20704_amd import api
    w = I.sedov_amr(nsteps=nsteps)
    say("fp64 parity: sedov amr, %d steps" % nsteps)
    T, D = build_both(w.ijkl, w.bc)
    got, dts = run_device(D, device_state(D, w.u), w.gamma, w.cfl, nsteps, api.RG_FP64)
    ref = T.permute_cells(w.u)
    ref_dts = T.run(ref, w.gamma, w.cfl, nsteps)
    worst, dmax = parity_metric(got, ref)
    say("  worst ratio %.3g, max |diff| %.3g" % (worst, dmax))
    assert worst <= 1e-12
    assert np.all(np.abs(dts - ref_dts) <= 1e-12 * ref_dts)


@pytest.mark.parametrize("case", small_trees(), ids=[c[0] for c in small_trees()])
def test_mixed_l1_and_conservation(case):
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = case
    u_in, gam = mk(ijkl)
    nsteps = 10
    say("mixed L1:", name)
    T, D = build_both(ijkl, bc)
    u0 = device_state(D, u_in)
    got, _ = run_device(D, u0, gam, 0.8, nsteps, api.RG_MIXED)
    ref = T.permute_cells(u_in)
    T.run(ref, gam, 0.8, nsteps)
    leaf, vol = leaf_and_volume(T)
    l1 = l1_rel(got, ref, leaf, vol)
    say("  L1 per field", l1)
    assert np.all(l1 <= 1e-5)
    if bc == I.PERIODIC:
        w = (vol * leaf)[:, None]
        tot0 = (w * T.permute_cells(u_in)).sum(0)
        tot = (w * got).sum(0)
        scale = (w * np.abs(got)).sum(0)
        assert np.all(np.abs(tot - tot0) <= 64 * nsteps * np.finfo(float).eps * scale)


def test_mixed_sedov_amr_l1():
    from paper_2607_20704_amd import api
    w = I.sedov_amr(nsteps=10)
    say("mixed L1: sedov amr, 10 steps")
    T, D = build_both(w.ijkl, w.bc)
    got, _ = run_device(D, device_state(D, w.u), w.gamma, w.cfl, 10, api.RG_MIXED)
    ref = T.permute_cells(w.u)
    T.run(ref, w.gamma, w.cfl, 10)
    leaf, vol = leaf_and_volume(T)
    l1 = l1_rel(got, ref, leaf, vol)
    say("  L1 per field", l1)
    assert np.all(l1 <= 1e-5)


@pytest.mark.parametrize("form", [0, 1])
def test_variants_are_bit_identical(form):
    """Every workgroup shape gives the same bits (the tuner cannot change
    results), and two runs give the same bits."""
    name, ijkl, bc, mk = small_trees()[2]
    u_in, gam = mk(ijkl)
    say("variants:", name, "form", form)
    T, D = build_both(ijkl, bc)
    u0 = device_state(D, u_in)
    outs = [run_device(D, u0, gam, 0.8, 4, form, tune=t)[0] for t in TUNINGS]
    again = run_device(D, u0, gam, 0.8, 4, form, tune=TUNINGS[0])[0]
    for o in outs[1:] + [again]:
        assert np.array_equal(o, outs[0])


def test_rebuild_every_step_matches_prebuilt():
    from paper_2607_20704_amd import api
    name, ijkl, bc, mk = small_trees()[3]
    u_in, gam = mk(ijkl)
    say("rebuild:", name)
    T, D = build_both(ijkl, bc)
    u0 = device_state(D, u_in)
    a = run_device(D, u0, gam, 0.8, 3, api.RG_FP64, rebuild=False)[0]
    b = run_device(D, u0, gam, 0.8, 3, api.RG_FP64, rebuild=True)[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("form", [0, 1])
def test_full_size_random_box_sampled(form):
    """256^3 periodic random-field box (2,097,152 octs) in the launch shape the
    benchmark uses: one device step, compared with the oracle's update of a
    sample of 3000 octs spread over the box (same dt)."""
    from paper_2607_20704_amd import api
    w = I.random_uniform()
    say("full size 256^3, form %d: building" % form)
    D = api.DeviceTree(w.ijkl, w.bc)
    T = O.Tree(w.ijkl, w.bc)
    assert np.array_equal(D.keys.cpu().numpy(), T.keys)
    assert np.array_equal(D.nbr27.cpu().numpy(), T.nbr27)
    u0 = device_state(D, w.u)
    u1 = torch.empty_like(u0)
    dt = D.step(u0, u1, w.gamma, w.cfl, form=form)
    torch.cuda.synchronize()
    ref0 = T.permute_cells(w.u)
    dt_ref = T.cfl_dt(ref0, w.gamma, w.cfl)
    assert dt.cpu().numpy()[0] == dt_ref
    rng = np.random.default_rng(77)
    sample = np.unique(np.concatenate([rng.integers(0, T.n, 2990), [0, 1, T.n - 1, T.n - 2]]))
    got = u1.cpu().numpy().reshape(-1, 8, 5)[sample].reshape(-1, 5)
    ref = np.zeros_like(ref0)
    corr = np.zeros(1)
    for o in sample:
        O.hydro_octs(T.ijkl, T.nbr27, T.son_mask, int(o), int(o) + 1, ref0, ref, corr, dt_ref, w.gamma)
    ref = ref.reshape(-1, 8, 5)[sample].reshape(-1, 5)
    if form == 0:
        worst, dmax = parity_metric(got, ref)
        say("  fp64 worst ratio %.3g, max |diff| %.3g" % (worst, dmax))
        assert worst <= 1e-12
    else:
        rel = np.abs(got - ref).sum(0) / np.abs(ref).sum(0)
        say("  mixed one-step relative L1 on the sample", rel)
        assert np.all(rel <= 1e-6)


BRICK_CASES = [
    ("sod_l5_outflow", lambda: (I.uniform_tree(5), I.OUTFLOW, lambda t: (I.sod_state(t, 1.4), 1.4))),
    ("random_l5_periodic", lambda: (I.uniform_tree(5), I.PERIODIC,
                                    lambda t: (I.grid_to_tree_state(t, 5, I.random_fields_grid(32, 31), 5 / 3), 5 / 3))),
    ("random_l6_periodic", lambda: (I.uniform_tree(6), I.PERIODIC,
                                    lambda t: (I.grid_to_tree_state(t, 6, I.random_fields_grid(64, 33), 5 / 3), 5 / 3))),
    ("sedov_l4_l6", lambda: (I.sedov_amr(base=4, lmax=6).ijkl, I.PERIODIC, lambda t: (I.sedov_state(t, 1.4), 1.4))),
    ("sphere_5_6_outflow", lambda: (I.sphere_tree(5, 6, (0.3, 0.6, 0.55), 0.2, I.OUTFLOW), I.OUTFLOW,
                                    lambda t: (I.grid_to_tree_state(t, 5, I.random_fields_grid(32, 32), 5 / 3), 5 / 3))),
]


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("case", BRICK_CASES, ids=[c[0] for c in BRICK_CASES])
def test_brick_schedule_bit_identical(case, form):
    """The brick kernel (complete 8^3-oct bricks, plane sweep) and the per-oct
    kernel give the same bits; FP64 also matches the oracle.  On the complete
    periodic levels the bricks go two by two along z by default; one by one
    they give the same bits."""
    name, mk = case
    ijkl, bc, state = mk()
    u_in, gam = state(ijkl)
    say("bricks:", name, "form", form)
    T, D = build_both(ijkl, bc)
    counts = D.schedule_counts()
    say("  schedule", counts)
    assert sum(c[0] for c in counts.values()) > 0
    u0 = device_state(D, u_in)
    a = run_device(D, u0, gam, 0.8, 5, form)[0]
    b = run_device(D, u0, gam, 0.8, 5, form, tune=(4, 256, 1))[0]
    diff = np.abs(a - b).max()
    say("  max |bricks - per-oct| = %.3g" % diff)
    assert np.array_equal(a, b)
    # the brick kernel compiled for another register budget (spilling or not)
    for waves in ((2, 3) if form == 0 else (3, 4)):
        c = run_device(D, u0, gam, 0.8, 5, form, tune=(4, 256, 0, 0, waves))[0]
        assert np.array_equal(a, c), waves
    # sibling groups left to the per-oct kernel, or on other workgroup sizes;
    # bricks one by one instead of in pairs (where pairs apply)
    for t in ((4, 256, 0, 0, 0, 1), (4, 256, 0, 0, 0, 0, 256), (4, 256, 0, 0, 0, 0, 384),
              (4, 256, 0, 0, 0, 0, 0, 1)):
        c = run_device(D, u0, gam, 0.8, 5, form, tune=t)[0]
        assert np.array_equal(a, c), t
    if form == 0:
        ref = T.permute_cells(u_in)
        T.run(ref, gam, 0.8, 5)
        worst, dmax = parity_metric(a, ref)
        say("  vs oracle: worst ratio %.3g, max |diff| %.3g" % (worst, dmax))
        assert worst <= 1e-12


@pytest.mark.parametrize("case", BRICK_CASES[3:], ids=[c[0] for c in BRICK_CASES[3:]])
def test_sibling_group_lists(case):
    """Per level above lmin, the group list holds exactly the octs outside
    bricks whose key ends in 0 (binary 000) and whose 7 following keys are
    its siblings; the single list the other octs outside bricks."""
    from paper_2607_20704_amd import api
    name, mk = case
    ijkl, bc, _ = mk()
    D = api.DeviceTree(ijkl, bc)
    keys = D.keys.cpu().numpy()
    lists = D.schedule_lists()
    total = 0
    for l in range(D.lmin, D.lmax + 1):
        bricks, rest, border, groups, singles = lists[l]
        e = int(D.level_begin[l + 1])
        want = [o for o in rest if l > D.lmin and keys[o] % 8 == 0 and o + 7 < e and keys[o + 7] == keys[o] + 7]
        assert np.array_equal(groups, np.array(want, dtype=groups.dtype)), l
        grouped = np.zeros(D.n, bool)
        for o in want:
            grouped[o:o + 8] = True
        assert grouped[rest].sum() == 8 * len(want)
        assert np.array_equal(singles, rest[~grouped[rest]]), l
        total += len(want)
    say("  %s: sibling groups %d" % (name, total))
    assert total > 0


@pytest.mark.parametrize("case", BRICK_CASES[3:], ids=[c[0] for c in BRICK_CASES[3:]])
def test_border_lists_and_unscheduled_corrections(case):
    """The schedule's per-level border lists (octs with a coarse cell across
    a face, which the scheduled step corrects from) equal a brute-force scan
    of the neighbour lists, and the step without a schedule (corrections
    over every oct above lmin) gives the same bits."""
    from paper_2607_20704_amd import api
    name, mk = case
    ijkl, bc, state = mk()
    u_in, gam = state(ijkl)
    D = api.DeviceTree(ijkl, bc)
    nbr = D.nbr27.cpu().numpy()
    lst = D.sched_list.cpu().numpy()
    face = nbr[:, [12, 14, 10, 16, 4, 22]]
    border = np.any((face < 0) & (face != O.OUTSIDE), axis=1)
    total = 0
    for l in range(D.lmin + 1, D.lmax + 1):
        b, e = int(D.level_begin[l]), int(D.level_begin[l + 1])
        want = b + np.nonzero(border[b:e])[0]
        got = lst[D.sched.border_begin[l]:D.sched.border_begin[l] + D.sched.border_count[l]]
        assert np.array_equal(got, want), l
        total += len(want)
    say("  border octs", total, "of", D.n - int(D.level_begin[D.lmin + 1]))
    assert total > 0
    U = api.DeviceTree(ijkl, bc, schedule=False)
    for form in (0, 1):
        a = run_device(D, device_state(D, u_in), gam, 0.8, 4, form)[0]
        c = run_device(U, device_state(U, u_in), gam, 0.8, 4, form)[0]
        assert np.array_equal(a, c), form


CHAIN_CASES = small_trees() + [
    ("sedov_l4_l6", I.sedov_amr(base=4, lmax=6).ijkl, I.PERIODIC, lambda t: (I.sedov_state(t, 1.4), 1.4)),
    ("deep_amr_l4_l7", I.deep_amr(base=4, lmax=7, nclump=60, sigma_a=2.0).ijkl, I.PERIODIC,
     lambda t: (I.deep_amr(base=4, lmax=7, nclump=60, sigma_a=2.0).u, 5.0 / 3.0)),
]


@pytest.mark.parametrize("tune", [None, (4, 256, 1)], ids=["bricks", "per_oct"])
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("case", CHAIN_CASES, ids=[c[0] for c in CHAIN_CASES])
def test_chained_dt_equals_separate_pass(case, form, tune):
    """The time step folded into the update (leaf cells without a split face
    neighbour) plus the corrected coarse cells equals, bit for bit, the
    separate CFL pass over the finished state: chained and unchained runs
    give identical states and time steps."""
    name, ijkl, bc, mk = case
    u_in, gam = mk(ijkl)
    say("chained dt:", name, "form", form, "tune", tune)
    from paper_2607_20704_amd import api
    D = api.DeviceTree(ijkl, bc)
    u0 = device_state(D, u_in)
    a, da = D.run(u0, gam, 0.8, 6, form=form, tune=tune)
    b, db = D.run(u0, gam, 0.8, 6, form=form, tune=tune, chain=True)
    torch.cuda.synchronize()
    assert np.array_equal(da.cpu().numpy(), db.cpu().numpy()), (da, db)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
